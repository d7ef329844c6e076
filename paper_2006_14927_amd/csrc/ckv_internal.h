// Internal definitions shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ckv.h"

namespace ckv {

// physical constants (CODATA 2018) in m, ns, MeV
constexpr double kSpeedOfLight = 0.299792458;      // m / ns
constexpr double kFineStructure = 7.2973525693e-3;
constexpr double kMassElectron = 0.51099895000;     // MeV
constexpr double kMassMuon = 105.6583755;           // MeV
constexpr double kPi = 3.14159265358979323846;

// Bunch-path launch geometry.
constexpr int kWave = 64;              // CDNA wavefront
constexpr int kMaxTileSegs = 64;       // steps per tile (one per lane at most)
constexpr int kStageBlock = 256;       // staging slots a wave claims at once
constexpr int kRunBlock = 256;         // run slots a wave claims at once
constexpr int kMaxEmitGrid = 512;      // bound on bunch-kernel workgroups (workspace sizing)
constexpr int kMaxEmitWaves = 16;     // waves per bunch-kernel workgroup
constexpr int kRowBlock = 64;          // tiles per block of the per-telescope scan
// Candidate grids are stacked in levels; level l lists, per cell, the spheres a
// line through the cell with observed w >= kGridWLevel[l] can meet (reach R/w).
constexpr int kGridLevels = 3;
constexpr double kGridWLevel[kGridLevels] = {0.2, 0.5, 0.85};
constexpr double kGridWLo = kGridWLevel[0];  // below it every sphere is tested

// Layout of one cell of the FP32 table: psi_i, psi_{i+1}-psi_i, P1_i..P5_i, 0.
constexpr int kCell32 = 8;
// Layout of one node of the FP64 table: psi_i, P1_i..P5_i.
constexpr int kNode64 = 6;

// Staging entry written by the bunch kernel for every sphere crossing (48 bytes:
// the record and what places it: tile, telescope, rank inside the tile, bunch).
struct alignas(16) StageEntry {
    float rec[8];        // dx, dy, u_o, v_o, t, h_e, photons, lambda
    uint32_t tile;       // emit tile
    uint32_t tel_sidx;   // telescope | (step index inside the tile) << 16
    uint32_t rank;       // index among this tile's crossings of this telescope
    uint32_t k;          // bunch index in the step (< 2^30: a tile holds fewer bunches)
};
static_assert(sizeof(StageEntry) == 48, "staging entry is 48 bytes");

// A tile's crossings per telescope are kept as runs, one per telescope the tile's
// bunches crossed: (telescope << kRunTelShift) | count, ascending telescope; the
// finalize replaces each count by the crossings of the same (shower, telescope)
// in earlier tiles.
constexpr int kRunTelShift = 40;
constexpr int64_t kRunValueMask = ((int64_t)1 << kRunTelShift) - 1;

// Control block in the workspace (zeroed by the first kernel of a run).  The
// counters every wave claims from (tiles, staging blocks, run blocks, screening
// tiles) sit on cache lines of their own: same-line atomics from all waves would
// serialise in one L2 channel.
enum CtrlSlot {
    kTileCounter = 0,   // next tile to claim (the mixed bunch kernel: tiles claimed past
                        // each wave's first, the next being the grid's wave count plus this)
    kBlockCounter = 32, // next staging block to claim
    kRunCounter = 64,   // next run block to claim
    kScreenCounter = 96,  // as kTileCounter, for the soft response's screening pass (the
                          // FP64 tile forward that may follow claims from kTileCounter)
    kNumTiles = 128,    // tiles of this run
    kNumRowBlocks,      // row blocks of the per-telescope scan
    kHits,              // crossings found
    kBunches,           // bunches generated
    kEmitting,          // steps with light
    kFirstLost,         // smallest tile with a crossing that found no staging or run slot
                        // (set to the tile count by the first kernel)
    kCutTile,           // tiles [0, kCutTile) are written
    kCutBlocks,         // row blocks holding them
    kRecords,           // their crossings
    kDrop0,             // CKV_N_DROP drop counters follow
    kCtrlSlots = kDrop0 + CKV_N_DROP + 4
};

}  // namespace ckv

struct ckv_atmo {
    int device = 0;
    int64_t n_nodes = 0;
    double h_obs = 0, step = 0, inv_step = 0, h_top = 0;
    double n_obs = 1;                // sqrt(1 + psi_0)
    std::vector<double> psi;         // host, n_nodes
    std::vector<double> P;           // host, 5 x n_nodes
    double psi_min = 0, psi_max = 0; // range of psi over the nodes
    bool psi_falls = false;          // psi non-increasing with altitude at every node
    double* d_node64 = nullptr;      // device, n_nodes x kNode64
    float* d_cell32 = nullptr;       // device, (n_nodes - 1) x kCell32
    std::vector<double> depth;       // host, n_nodes, vertical depth [g/cm^2]; empty: none
    double* d_depth = nullptr;       // device copy of depth
    // node tables (non-uniform altitudes, binary-search lookups); empty: uniform grid
    std::vector<double> h_nodes;     // host, n_nodes
    double* d_hnodes = nullptr;      // device: n_nodes altitudes, then n_nodes-1 inverse widths
};

// Candidate grid: cells of size `cell` starting at (gx0, gy0); the list of
// cell c holds, in ascending order, every telescope whose (effective) sphere
// can be met by a line through a ground point in c with observed w >= kGridWLo.
struct ckv_grid {
    double gx0 = 0, gy0 = 0, cell = 1, inv_cell = 1;
    int32_t nx = 0, ny = 0;
    int32_t level_cells = 0;         // nx*ny
    std::vector<int32_t> cell_off;   // kGridLevels*nx*ny + 1, level-major
    std::vector<uint16_t> cell_list;
    // per cell, packed: {offset into cell_list, count | first listed sphere << 16},
    // so a bunch learns its first candidate with the one load that finds its cell
    std::vector<uint32_t> cell_ent;  // 2 x kGridLevels*nx*ny
    int32_t* d_cell_off = nullptr;
    uint16_t* d_cell_list = nullptr;
    uint32_t* d_cell_ent = nullptr;
};

struct ckv_array {
    int device = 0;
    int32_t n_tel = 0;
    std::vector<double> x, y, r;
    double* d_tel = nullptr;         // device, n_tel x 4: X, Y, R, R^2
    ckv_grid hit;                    // radii R (sphere crossings)
    ckv_grid soft;                   // radii sqrt(R^2 + 2 R sigma z_cut) + margin (soft response)
    double soft_sigma = 0;           // 0: no soft grid
    double screen_rmax = 0;          // largest screening radius (R_s of d_tel_screen)
    double* d_tel_screen = nullptr;  // device, n_tel x 4: X, Y, R_s, R_s^2 with R_s the soft
                                     // cut radius plus kScreenMargin (screening pass)
};

namespace ckv {

void set_error(const std::string& msg);

// host builders (ckv_tables.cpp)
int build_atmo_tables(const double* alt, const double* eta, int64_t n, double h_obs, double step,
                      ckv_atmo* a);
// tables on the input's own altitudes above h_obs (node tables)
int build_node_tables(const double* alt, const double* eta, int64_t n, double h_obs, ckv_atmo* a);
// psi_min, psi_max and psi_falls of a's node values
void psi_range(ckv_atmo* a);
// depth at the nodes of a (after build_atmo_tables), the same interpolation as eta
void build_depth_table(const double* alt, const double* depth, int64_t n, ckv_atmo* a);
int build_array_grid(const ckv_array* arr, const std::vector<double>& radius, ckv_grid* g);
constexpr double kSoftZCut = 40.0;   // Phi(-40) underflows to exactly 0 in FP64
// margin of the soft response's screening spheres over the cut radius [m]
constexpr double kScreenMargin = 0.01;
// Bound of the mixed path's ground-point error per metre of height above the
// observation level: e_g = dh (kScreenErrDir (1/w + 1/w^2) + kScreenErrSeries / w^3).
// The first term: the FP32 cone vector carries an absolute direction error below
// sin(theta_c) x 3e-7 <= 7.3e-9 (theta_c <= 1.4 deg at n - 1 <= 3e-4), which
// moves the ground point by dh delta (1/w + |u|/w^2).  The second: the FP32 series
// corrections, below 2^-20 relative of q D1/2 <= (1/w^2) 3e-4 dh, moved by u/w.
// Screened bunches whose bound passes half the margin are listed unconditionally.
constexpr double kScreenErrDir = 1e-8;
constexpr double kScreenErrSeries = 5e-10;
int param_spec_check(const ckv_atmo_param_spec* sp, const double* theta);
void param_profile(const ckv_atmo_param_spec* sp, const double* theta, std::vector<double>* alt,
                   std::vector<double>* eta);
void param_backward(const ckv_atmo_param_spec* sp, const double* theta, const ckv_atmo* a,
                    const double* g_psi, const double* g_P, double* g_theta);



// kernel launchers (ckv_kernels.hip)
struct RunPlan {
    // inputs
    ckv_segments segs;
    ckv_showers showers;
    ckv_params params;
    const ckv_atmo* atmo;
    const ckv_array* arr;
    ckv_output out;
    hipStream_t stream;
    // derived
    int32_t tile_segs;
    int64_t max_tiles, max_row_blocks, stage_slots;
    int32_t emit_grid, emit_waves;
    int32_t prof_bins;          // longitudinal-profile bins, 0 = no profile
    double k_ft;
    ckv_cursor cursor;          // first step of the run (step 0, shower 0 without one)
    int64_t run_cap;            // run slots
    // workspace carve-out
    int64_t* ctrl;
    ckv_result* ws_result;      // report of the soft entry points when the caller has none
    int64_t* tiles_before;      // n_showers + 1
    int64_t* blocks_before;     // n_showers + 1
    int64_t* shower_first;      // n_showers: first step of each shower in this run
    int64_t* tile_run_off;      // max_tiles: first run of the tile
    int32_t* tile_run_n;        // max_tiles: runs of the tile
    int32_t* tile_hits;         // max_tiles: crossings of the tile
    int64_t* runs;              // run_cap
    int32_t* block_sums;        // n_tel x max_row_blocks (telescope-major)
    int64_t* block_hits;        // max_row_blocks: crossings per row block
    int32_t* shower_tel;        // n_showers x n_tel
    int32_t* stage_fill;        // stage_slots / kStageBlock
    StageEntry* stage;          // stage_slots
};

size_t workspace_layout(int64_t n_segments, int32_t n_showers, int32_t n_tel, int64_t capacity,
                        const ckv_params* p, RunPlan* plan, void* base);
// ckv_run after its handle-free checks: validates, lays out `workspace` and launches
int run_checked(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                const ckv_atmo* atmo, const ckv_array* arr, void* workspace, size_t ws_bytes,
                ckv_output* out, const ckv_cursor* resume_from, void* stream);
// bunch-kernel workgroups of a launch with params->grid == 0 on the current device
int default_emit_grid(int* grid);
int launch_run(RunPlan& plan);
int launch_count(const ckv_segments* segs, const ckv_params* p, const ckv_atmo* atmo, double k_ft,
                 int64_t* n_b, hipStream_t stream);
// waves per bunch-kernel workgroup (at most max_waves) and its LDS bytes
int emit_config(int precision, int n_tel, int prof_bins, const ckv_atmo* atmo, int tile_segs,
                int max_waves, int* waves, size_t* lds_bytes, bool narrow_ok);

struct SoftPlan {
    const int64_t* n_b_frozen;
    double sigma;
    const double* gS;       // backward: dL/dS per (shower, telescope)
    const double* gA;       // backward: dL/dA
    double* S;              // forward outputs
    double* A;
    double* g_psi;          // backward outputs (n_nodes)
    double* g_P;            // backward outputs (5 x n_nodes)
    uint64_t* ids;          // bunch list (NULL: none)
    int64_t ids_cap;
    int64_t* ids_count;
};
int launch_soft(RunPlan& plan, const SoftPlan& sp, int mode);

}  // namespace ckv
