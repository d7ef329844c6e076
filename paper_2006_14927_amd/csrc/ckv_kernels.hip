// HIP kernels of the Cherenkov photon-bunch path for gfx950 (CDNA4).
//
// Pipeline of one run (all on the caller's stream, no host synchronisation):
//   init      - zero the control block, validate shower offsets, count tiles
//               (a tile = up to tile_segs consecutive steps of one shower);
//   emit      - persistent: each wavefront claims tiles; per tile it computes
//               the step setups (FP64, one step per lane: photon yield, bunch
//               count, Cherenkov angle, frame), scans the bunch counts across
//               the wave, then walks the tile's bunches 64 at a time (one per
//               lane): Philox draws, sub-step emission point, direction on the
//               cone, LDS-staged atmosphere tables, refraction series, ground
//               point, candidate spheres, and records every crossing in a
//               staging area together with its rank among the tile's crossings
//               of the same telescope;
//   finalize  - per-telescope prefix sums over tiles, CSR offsets per
//               (shower, telescope), and a scatter of the staged records to
//               their final slots (ascending step, then bunch).
// Paper mapping: App. A (steps -> photon count -> bunches of ~5 photons, one
// per sub-step -> propagation -> telescope output), App. B (observed
// direction, displacement, travel time), sec. 3.3.2 (uniform fine tables).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <set>
#include <type_traits>
#include <utility>

#include "ckv_internal.h"

namespace ckv {

// --------------------------------------------------------------------------
// kernel arguments
// --------------------------------------------------------------------------
struct Args {
    const double *x0, *y0, *h0, *u, *v, *w, *len, *t0, *energy;
    const uint8_t* ptype;
    int64_t n;
    const uint32_t* step_id;    // counter word 1 per step, or NULL
    const int64_t* seg_offsets;
    const double* t_ref;
    const uint32_t* shower_ids;
    const int64_t* seg_id_base;
    int32_t n_showers;
    // atmosphere
    int32_t n_nodes;
    double h_obs, step, inv_step, h_top, n_obs;
    const double* node64;
    const float* cell32;
    int32_t lds_entries;        // table entries staged in LDS (the rest read from HBM)
    // node tables (binary-search lookups): n_nodes altitudes then n_nodes-1 inverse
    // widths; NULL for the uniform grid
    const double* hnodes;
    int32_t search_pow2;        // largest power of two below n_nodes - 1
    // longitudinal profile (prof_bins = 0: none)
    const double* depth;        // n_nodes, vertical depth [g/cm^2]
    double* prof_ph;            // n_showers x prof_bins
    int64_t* prof_bu;
    double inv_bin;
    int32_t prof_bins;
    // telescopes and candidate grid
    int32_t n_tel;
    const double* tel;          // X, Y, R, R^2
    double gx0, gy0, inv_cell;
    int32_t nx, ny, level_cells;
    const int32_t* cell_off;
    const uint16_t* cell_list;
    const uint2* cell_ent;      // per cell: {offset, count | first sphere << 16}
    // parameters
    double bunch_size, k_ft, inv_l1, dl, w_min;
    int32_t grazing_exact;      // 1: bunches with 0 < w <= w_min take propagate_exact
    double earth_r;             // > 0: spherical shells of this radius (curved variant)
    double r_obs;               // earth_r + h_obs
    uint32_t key0, key1;
    int32_t tile_segs;
    // first step of the run (a resume cursor; step 0 of shower 0 without one)
    int64_t cur_step;
    int32_t cur_shower;
    // workspace and output
    int64_t* ctrl;
    int64_t* tiles_before;
    int64_t* blocks_before;
    int64_t* shower_first;      // first step of each shower in this run
    int64_t* tile_run_off;
    int32_t* tile_run_n;
    int32_t* tile_hits;
    int64_t* runs;
    int64_t run_cap;
    int32_t* block_sums;        // telescope-major: block_sums[k * max_row_blocks + b]
    int64_t* block_hits;
    int32_t* shower_tel;
    int32_t* stage_fill;
    StageEntry* stage;
    int64_t stage_blocks;
    int64_t max_tiles;
    int64_t max_row_blocks;
    float* records;
    int64_t* ids;
    int64_t capacity;
    int64_t* tel_offsets;
    ckv_result* result;
    // screening pass of the soft response (kFeatScreen): frozen bunch counts and the
    // list of candidate bunches {ids, capacity, count}
    const int64_t* nb_frozen;
    uint64_t* list_ids;
    int64_t list_cap;
    int64_t* list_count;
    // the screening pass's per-step cull (cull_rmax = 0: off): the largest screening
    // radius; x0 = (psi_max - psi_min) / (1 + psi_min); b0 = x0 times the bound of
    // |1 - T4(x)| / |x| (1/2 for psi non-increasing with altitude, 4/5 otherwise); a
    // bound of (n_e / n_obs)^2
    double cull_rmax, cull_x0, cull_b0, cull_rho2;
};

// Memory accesses whose address space is explicit.  Where one access may go to LDS
// or to HBM, a generic pointer makes the compiler use one generic (flat)
// instruction for both, which costs every access, also the LDS ones; reads and
// atomics through these types keep the two kinds apart.
typedef float f32x4 __attribute__((ext_vector_type(4)));
using LdsF64 = __attribute__((address_space(3))) double;
using HbmF64 = __attribute__((address_space(1))) double;
using LdsF32x4 = __attribute__((address_space(3))) f32x4;
using HbmF32x4 = __attribute__((address_space(1))) f32x4;

__device__ __forceinline__ const LdsF64* as_lds(const double* p) { return (const LdsF64*)p; }
__device__ __forceinline__ const HbmF64* as_hbm(const double* p) { return (const HbmF64*)p; }
__device__ __forceinline__ const LdsF32x4* as_lds4(const float* p) { return (const LdsF32x4*)p; }
__device__ __forceinline__ const HbmF32x4* as_hbm4(const float* p) { return (const HbmF32x4*)p; }

__device__ __forceinline__ void lds_add(double* p, double v)
{
    __hip_atomic_fetch_add((LdsF64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void hbm_add(double* p, double v)
{
    __hip_atomic_fetch_add((HbmF64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------------------
// wave helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// x of the lane the DPP control CTRL names as source, in the rows ROWS enables; 0
// where there is no source or the row is masked off
template <int CTRL, int ROWS>
__device__ __forceinline__ int64_t dpp_take(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)x >> 32), CTRL, ROWS,
                                                              0xf, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive sum of x over lanes 0..lane by DPP lane moves (no LDS round trips):
// shifts by 1, 2, 4 and 8 inside each row of 16 lanes, then lane 15 of rows 0 and 2
// into rows 1 and 3 (row_bcast:15), then lane 31 into rows 2 and 3 (row_bcast:31).
// Called by the whole wave.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t x)
{
    x += dpp_take<0x111, 0xf>(x);   // row_shr:1
    x += dpp_take<0x112, 0xf>(x);   // row_shr:2
    x += dpp_take<0x114, 0xf>(x);   // row_shr:4
    x += dpp_take<0x118, 0xf>(x);   // row_shr:8
    x += dpp_take<0x142, 0xa>(x);   // row_bcast:15
    x += dpp_take<0x143, 0xc>(x);   // row_bcast:31
    return x;
}

// The same by lane shuffles (LDS round trips, fewer registers): the mixed
// kernel's called tile setup, where the DPP form's registers cost the bunch loop.
__device__ __forceinline__ int64_t wave_incl_scan_shfl(int64_t x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    return x;
}

// x of lane 63 (a register read, not an LDS round trip)
__device__ __forceinline__ int64_t wave_last(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), kWave - 1);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Smallest x over the lanes where it is below `none` (at least one lane is):
// take the first such lane's value and repeat while a lane holds a smaller one.
// Passes = distinct values below the result + 1, usually one or two; ballots
// and lane reads only, no LDS round trips.
__device__ __forceinline__ int wave_min_sparse(int x, int none)
{
    uint64_t below = __ballot(x < none);
    int m = none;
    while (below) {
        m = __builtin_amdgcn_readlane(x, __builtin_ctzll(below));
        below = __ballot(x < m);
    }
    return m;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T uniform(T x)
{
    return __shfl(x, 0);
}

// A value every lane holds alike, made visibly uniform to the compiler (a scalar
// register), so that control flow depending on it stays scalar.
__device__ __forceinline__ int64_t scalar64(int64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Candidate-grid level for a line with observed w^2 = wo2 (>= kLevelW2[0]):
// the deepest level whose w floor the line clears, with a 1e-6 margin that
// covers the rounding of wo2.
constexpr double kLevelW2[kGridLevels] = {
    kGridWLevel[0] * kGridWLevel[0] + 1e-6, kGridWLevel[1] * kGridWLevel[1] + 1e-6,
    kGridWLevel[2] * kGridWLevel[2] + 1e-6};
static_assert(kGridLevels == 3, "grid_level selects among three levels");

__device__ __forceinline__ int grid_level(double wo2)
{
    return wo2 >= kLevelW2[2] ? 2 : (wo2 >= kLevelW2[1] ? 1 : 0);
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers applied to
// words 0 and 2, key advanced by the Weyl constants between rounds.
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t r[4])
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    r[0] = c0; r[1] = c1; r[2] = c2; r[3] = c3;
}

// --------------------------------------------------------------------------
// Step setup, FP64, without FMA contraction: the bunch count must come out of
// exactly these IEEE operations.  App. A: photons per step, split into
// bunches of about bunch_size photons, one per equal sub-step.
// --------------------------------------------------------------------------
struct Setup {
    int status;        // -1: emits light; otherwise CKV_DROP_*
    int64_t nb;
    double photons, cos_t, sin_t, ds, inv_bc;
    double b1x, b1y, b1z, b2x, b2y, b2z;
    double x0, y0, h0, t0, u, v, w;   // the step's inputs as loaded (for its record)
};

__device__ __forceinline__ double psi_fp64(const Args& a, double h)
{
#pragma clang fp contract(off)
    double hc = h < a.h_obs ? a.h_obs : (h > a.h_top ? a.h_top : h);
    int64_t i;
    double f;
    if (a.hnodes) {
        // node tables: binary search for the bracketing pair, then the fraction
        int lo = 0, hi = a.n_nodes - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.hnodes[mid] <= hc) lo = mid; else hi = mid;
        }
        i = lo;
        f = (hc - a.hnodes[lo]) / (a.hnodes[lo + 1] - a.hnodes[lo]);
    } else {
        double x = (hc - a.h_obs) * a.inv_step;
        i = (int64_t)floor(x);
        if (i > a.n_nodes - 2) i = a.n_nodes - 2;
        f = x - (double)i;
    }
    double lo = a.node64[kNode64 * i], hi = a.node64[kNode64 * (i + 1)];
    return lo + f * (hi - lo);
}

// Curved variant: x, y horizontal at the array origin, z along the origin's
// vertical from sea level, the Earth's centre at (0, 0, -R).  The altitude of a
// point is its distance from the centre minus R, written without the
// cancellation of sqrt(...) - R; no contraction, so drop decisions and table
// cells match the FP64 definition's operations.
__device__ __forceinline__ double curved_altitude(double R, double x, double y, double z)
{
#pragma clang fp contract(off)
    const double q = x * x + y * y;
    const double rz = R + z;
    const double r = sqrt(q + rz * rz);
    return (q + z * (2.0 * R + z)) / (r + R);
}

__device__ __forceinline__ void step_setup(const Args& a, int64_t i, Setup& st)
{
#pragma clang fp contract(off)
    st.nb = 0;
    st.status = -1;
    const double x0 = a.x0[i], y0 = a.y0[i], h0 = a.h0[i];
    const double u = a.u[i], v = a.v[i], w = a.w[i];
    const double L = a.len[i], t0 = a.t0[i], E = a.energy[i];
    const double m = a.ptype[i] == CKV_MUON ? kMassMuon : kMassElectron;
    st.x0 = x0; st.y0 = y0; st.h0 = h0; st.t0 = t0; st.u = u; st.v = v; st.w = w;
    // (E c with c = m / 1 GeV in (0, 1) is finite exactly when E is; testing it, with
    // every test evaluated (no short circuit), puts all the step's loads in one round)
    const int n_finite = (int)isfinite(x0) + (int)isfinite(y0) + (int)isfinite(h0) + (int)isfinite(u) +
                         (int)isfinite(v) + (int)isfinite(w) + (int)isfinite(L) + (int)isfinite(t0) +
                         (int)isfinite(E * (m * 1e-3));
    const bool finite = n_finite == 9;
    if (!finite || !(L > 0.0)) { st.status = CKV_DROP_NONFINITE; return; }
    const double r = m / E;
    const double r2 = r * r;                           // 1 - beta^2
    if (!(r2 < 1.0)) { st.status = CKV_DROP_MASS; return; }
    double h_mid;                                      // index at the step midpoint
    if (a.earth_r > 0.0) {
        const double hl = 0.5 * L;
        h_mid = curved_altitude(a.earth_r, x0 + hl * u, y0 + hl * v, h0 - hl * w);
    } else {
        h_mid = h0 - (0.5 * L) * w;
    }
    const double psi = psi_fp64(a, h_mid);
    const double n2 = 1.0 + psi;
    const double num = psi - n2 * r2;                  // beta^2 n^2 - 1
    if (!(num > 0.0)) { st.status = CKV_DROP_THRESHOLD; return; }
    const double sin2 = num / (n2 * (1.0 - r2));       // sin^2 of the Cherenkov angle
    const double N = (a.k_ft * L) * sin2;              // Frank-Tamm photon count
    const double nbd = ceil(N / a.bunch_size);
    st.nb = (int64_t)nbd;
    st.photons = N / nbd;
    st.cos_t = 1.0 / sqrt((1.0 - r2) * n2);           // 1 / (beta n)
    st.sin_t = sqrt(sin2);
    st.ds = L / nbd;
    st.inv_bc = 1.0 / (sqrt(1.0 - r2) * kSpeedOfLight);
    // orthonormal frame around D = (u, v, -w) (Duff et al., JCGT 2017)
    const double Dx = u, Dy = v, Dz = -w;
    const double sgn = copysign(1.0, Dz);
    const double ia = -1.0 / (sgn + Dz);
    const double ib = Dx * Dy * ia;
    st.b1x = 1.0 + sgn * Dx * Dx * ia;
    st.b1y = sgn * ib;
    st.b1z = -sgn * Dx;
    st.b2x = ib;
    st.b2y = sgn + Dy * Dy * ia;
    st.b2z = -Dy;
}

// --------------------------------------------------------------------------
// sin and cos of 2 pi (r + 1/2) / 2^32 from the integer draw r, in turns.
// Mixed path: the hardware sine and cosine, which take their argument in turns:
// the quadrant from the top two bits, the angle inside it as an FP32 number of
// turns in [0, 1/4) (rounding below 1e-7 rad); errors near 1e-7, i.e. ~2e-9 in
// the photon direction once scaled by sin(theta_c) < 0.03.  The quadrant's
// rotation, (s, c) = (sq, cq), (cq, -sq), (-sq, -cq), (-cq, sq) for q = 0..3, is
// a swap on bit 30 of r and sign flips on bit 31 (sine) and on bit 31 of
// r + 2^30 (cosine).
// --------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns_hw(uint32_t r, float& s, float& c)
{
    const float t = fmaf((float)(r & 0x3FFFFFFFu), 2.3283064365386963e-10f, 1.16415321826934814e-10f);
    const float sq = __builtin_amdgcn_sinf(t), cq = __builtin_amdgcn_cosf(t);
    const bool swap = (r & 0x40000000u) != 0;
    const uint32_t s0 = __float_as_uint(swap ? cq : sq), c0 = __float_as_uint(swap ? sq : cq);
    s = __uint_as_float(s0 ^ (r & 0x80000000u));
    c = __uint_as_float(c0 ^ ((r + 0x40000000u) & 0x80000000u));
}

// The same in FP64 for the FP64 path: quadrant and half-quadrant fold from the
// integer draw, then Taylor series of sin and cos on |a| <= pi/4 to a^17 and a^16
// (next terms below 1e-17).
__device__ __forceinline__ void sincos_turns64(uint32_t r, double& s, double& c)
{
    const uint32_t q = r >> 30;
    const uint32_t low = r & 0x3FFFFFFFu;
    const bool upper = low >= 0x20000000u;
    const uint32_t m = upper ? (0x3FFFFFFFu - low) : low;
    const double kq = 1.4629180792671596e-09;          // (pi/2) / 2^30
    const double a = fma((double)m, kq, 0.5 * kq);
    const double a2 = a * a;
    double sa = fma(a2, 1.0 / 355687428096000.0, -1.0 / 1307674368000.0);
    sa = fma(a2, sa, 1.0 / 6227020800.0);
    sa = fma(a2, sa, -1.0 / 39916800.0);
    sa = fma(a2, sa, 1.0 / 362880.0);
    sa = fma(a2, sa, -1.0 / 5040.0);
    sa = fma(a2, sa, 1.0 / 120.0);
    sa = fma(a2, sa, -1.0 / 6.0);
    sa = a * fma(a2, sa, 1.0);
    double ca = fma(a2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);
    ca = fma(a2, ca, 1.0 / 479001600.0);
    ca = fma(a2, ca, -1.0 / 3628800.0);
    ca = fma(a2, ca, 1.0 / 40320.0);
    ca = fma(a2, ca, -1.0 / 720.0);
    ca = fma(a2, ca, 1.0 / 24.0);
    ca = fma(a2, ca, -0.5);
    ca = fma(a2, ca, 1.0);
    const double cq = upper ? sa : ca;
    const double sq = upper ? ca : sa;
    c = (q == 0) ? cq : (q == 1) ? -sq : (q == 2) ? -cq : sq;
    s = (q == 0) ? sq : (q == 1) ? cq : (q == 2) ? -sq : -cq;
}

// 1/x in FP64 from the hardware reciprocal and two Newton steps (to an ulp or so,
// without the correctly rounded division's scaling sequence)
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// --------------------------------------------------------------------------
// LDS layout of the bunch kernel
//   [atmosphere table][wave 0 area][wave 1 area]...
// wave area: TS step entries (the emitting steps of the current tile,
// compacted), a 64-entry flag row used to map bunches to steps, the per-
// telescope crossing counters of the tile, and the wave's run counters.
// --------------------------------------------------------------------------
// Exact propagation of a grazing bunch (0 < w <= w_min), cell by cell in FP64
// from the FP64 node table, where the moment series is not used (sec. 4.3.1 and
// App. C: rare bunches take a slow path).  With Snell's invariant
// p = n_e sin(theta_e), s = n cos(theta) obeys s^2 = n_e^2 w^2 + psi - psi_e,
// linear inside a cell, and a cell of height dz between s_t (top) and s_b
// (bottom) adds 2 p dz / (s_t + s_b) to the horizontal advance and
// (2/3) dz (s_t^2 + s_t s_b + s_b^2) / (s_t + s_b) + 2 p^2 dz / (s_t + s_b)
// to c times the travel time; a downward ray never turns.
__device__ __forceinline__ void propagate_exact(const Args& a, double xe, double ye, double he,
                                             double u, double v, double w, double& xg, double& yg,
                                             double& T, double& ne)
{
    const double* nd = a.node64;
    const double x = (he - a.h_obs) * a.inv_step;
    int c = min((int)x, a.n_nodes - 2);
    const double f = x - (double)c;
    const double psi_e = nd[kNode64 * c] + f * (nd[kNode64 * (c + 1)] - nd[kNode64 * c]);
    const double ne2 = 1.0 + psi_e;
    ne = sqrt(ne2);
    const double sin_e = sqrt(u * u + v * v);
    const double p = ne * sin_e;
    const double s0sq = ne2 * w * w;
    double X = 0.0, cT = 0.0, h_top = he, s_t = sqrt(s0sq);
    for (int i = c; i >= 0; --i) {
        const double h_b = a.h_obs + (double)i * a.step;
        const double dz = h_top - h_b;
        const double s_b = sqrt(s0sq + (nd[kNode64 * i] - psi_e));
        if (dz > 0.0) {
            const double inv = 1.0 / (s_t + s_b);
            X += 2.0 * p * dz * inv;
            cT += (2.0 / 3.0) * dz * (s_t * s_t + s_t * s_b + s_b * s_b) * inv + 2.0 * p * p * dz * inv;
        }
        h_top = h_b;
        s_t = s_b;
    }
    xg = sin_e > 0.0 ? xe + (u / sin_e) * X : xe;
    yg = sin_e > 0.0 ? ye + (v / sin_e) * X : ye;
    T = cT / kSpeedOfLight;
}

// FP64 reciprocal square root: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// One Newton step on the hardware estimates (relative errors below 2^-23 for rsq
// and 2^-24 for rcp on this chip): ~1e-14 relative, for the per-cell factors of
// the curved tracer, where such errors stay far below the result's rounding.
__device__ __forceinline__ double rsqrt64_1(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

__device__ __forceinline__ double rcp64_1(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// Curved atmosphere: exact propagation through spherical shells (radius R =
// a.earth_r, centre (0, 0, -R)).  n depends on the altitude h = r - R only, so
// the ray stays in the plane of the centre, its emission point and direction,
// and keeps Bouguer's invariant K = n r sin(zeta) (zeta from the local
// vertical).  With s = sqrt(n^2 r^2 - K^2), the polar angle about the centre
// and the optical path down to the observation sphere r_obs are
//   theta = int K / (r s) dr,    c T = int n^2 r / s dr,
// integrated cell by cell (psi linear in h inside a cell).  s^2 is written
// relative to the emission point, s^2 = s_e^2 + (h - h_e)(r + r_e) + psi r^2 -
// psi_e r_e^2 with s_e = n_e r_e cos(zeta_e), which stays accurate for grazing
// rays.  Over a cell s^2 is nearly linear in h, so the substitution
// h = h_b + dh (u^2 - s_b^2) / (s_t^2 - s_b^2), u from s_b to s_t, turns
//   int F / s dh  into  dh / (s_t + s_b) * sum of F u / s at the 2-point
// Gauss-Legendre nodes of [s_b, s_t] (u / s is 1 up to the cell's curvature of
// s^2, ~1e-9, so two nodes reach FP64 rounding).  The ground point is the
// emission point's radial direction turned by theta towards the ray's tangential
// direction, at r_obs; the arrival direction has sin(zeta_g) = K / (n_obs r_obs).
// While n r grows with r (air at the Earth's radius: no ducting) the ray reaches
// the ground iff s^2 > 0 there, and one with cos(zeta_e) <= 0 never comes down.
// The upward and turning decisions use the FP64 definition's operations.
// Returns -1 (reached the ground), CKV_DROP_UPWARD or CKV_DROP_GRAZING.
__device__ __forceinline__ int propagate_curved(const Args& a, double xe, double ye, double ze,
                                                double he, double u, double v, double w,
                                                double& xg, double& yg, double& T, double& uo,
                                                double& vo)
{
    const double R = a.earth_r;
    const double* nd = a.node64;
    double rz, r_e, mu_num, psi_e, ne2, K, s2e, Mre, s2g;
    {
#pragma clang fp contract(off)
        rz = R + ze;
        r_e = sqrt(xe * xe + ye * ye + rz * rz);
        mu_num = w * rz - u * xe - v * ye;          // r_e cos(zeta_e), zeta_e from the downward vertical
        if (!(mu_num > 0.0)) return CKV_DROP_UPWARD;
        psi_e = psi_fp64(a, he);
        ne2 = 1.0 + psi_e;
        const double Lx = -ye * w - rz * v, Ly = rz * u + xe * w, Lz = xe * v - ye * u;
        K = sqrt(ne2) * sqrt(Lx * Lx + Ly * Ly + Lz * Lz);   // n_e |(P_e - C) x D|
        s2e = ne2 * (mu_num * mu_num);
        Mre = psi_e * r_e * r_e;
        s2g = s2e + ((a.h_obs - he) * (a.r_obs + r_e) + nd[0] * a.r_obs * a.r_obs - Mre);
        if (!(s2g > 0.0)) return CKV_DROP_GRAZING;
    }
    const double x = (he - a.h_obs) * a.inv_step;
    const int c = min((int)x, a.n_nodes - 2);
    constexpr double kg = 0.57735026918962576451;   // 1/sqrt(3)
    double theta = 0.0, opt = 0.0;
    double h_t = he, s2t = s2e, s_t = s2e * rsqrt64_1(s2e);
    for (int i = c; i >= 0; --i) {
        const double h_b = a.h_obs + (double)i * a.step;
        const double psi_b = nd[kNode64 * i];
        const double r_b = R + h_b;
        const double s2b = i == 0 ? s2g : s2e + ((h_b - he) * (r_b + r_e) + psi_b * r_b * r_b - Mre);
        const double s_b = s2b * rsqrt64_1(s2b);
        const double dh = h_t - h_b;
        if (dh > 0.0 && s2t != s2b) {    // (a cell of zero s^2 span adds ~dh/s: nothing)
            const double g = (nd[kNode64 * (i + 1)] - psi_b) * a.inv_step;   // dpsi/dh in the cell
            const double inv_ds2 = rcp64_1(s2t - s2b);
            const double inv_rb = rcp64_1(r_b);
            const double mid = 0.5 * (s_t + s_b), half = (0.5 * kg) * (s_t - s_b);
            double a_th = 0.0, a_op = 0.0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double uq = q ? mid + half : mid - half;
                const double xq = dh * ((uq * uq - s2b) * inv_ds2);     // h_q - h_b
                const double psq = fma(g, xq, psi_b);
                const double rq = r_b + xq;
                const double s2q = s2e + ((h_b + xq - he) * (rq + r_e) + psq * rq * rq - Mre);
                const double ratio = uq * rsqrt64_1(s2q);
                const double e = xq * inv_rb;                            // 1/r_q = (1 - e + e^2) / r_b
                a_th += ratio * (inv_rb * fma(e, e - 1.0, 1.0));
                a_op += ((1.0 + psq) * rq) * ratio;
            }
            const double scale = dh * rcp64_1(s_t + s_b);
            theta = fma(scale, K * a_th, theta);
            opt = fma(scale, a_op, opt);
        }
        h_t = h_b;
        s2t = s2b;
        s_t = s_b;
    }
    // ground point and arrival direction in the ray plane
    const double inv_re = rcp64(r_e);
    const double rho0 = xe * inv_re, rho1 = ye * inv_re, rho2 = rz * inv_re;
    const double mu = mu_num * inv_re;
    double t0 = fma(mu, rho0, u), t1 = fma(mu, rho1, v), t2 = fma(mu, rho2, -w);
    const double sz2 = t0 * t0 + t1 * t1 + t2 * t2;
    const double isz = sz2 > 0.0 ? rsqrt64(sz2) : 0.0;
    t0 *= isz; t1 *= isz; t2 *= isz;
    double sth, cth;
    sincos(theta, &sth, &cth);
    const double rg0 = cth * rho0 + sth * t0, rg1 = cth * rho1 + sth * t1;
    const double tg0 = cth * t0 - sth * rho0, tg1 = cth * t1 - sth * rho1;
    const double inv_nr = rcp64(a.n_obs * a.r_obs);
    const double sin_g = K * inv_nr, cos_g = s2g * rsqrt64(s2g) * inv_nr;
    xg = a.r_obs * rg0;
    yg = a.r_obs * rg1;
    uo = sin_g * tg0 - cos_g * rg0;
    vo = sin_g * tg1 - cos_g * rg1;
    T = opt * (1.0 / kSpeedOfLight);
    return -1;
}

// Depth bin of an emission altitude h_obs <= h < h_top, given its table cell c
// and fraction f (x = (h - h_obs) / step, c = floor(x), f = x - c): the depth
// table read like the index and binned by floor(X * (1/width)), in FP64
// without contraction, so the bin is the one the FP64 definition gives.
__device__ __forceinline__ int profile_bin(const Args& a, int c, double f)
{
#pragma clang fp contract(off)
    const double X = a.depth[c] + f * (a.depth[c + 1] - a.depth[c]);
    int b = (int)floor(X * a.inv_bin);
    b = max(0, min(b, a.prof_bins - 1));
    return b;
}

template <int PREC>
struct StepEntry;

// mixed: FP64 position/time/direction, FP32 perpendicular cone vectors
template <>
struct alignas(16) StepEntry<1> {
    double x0, y0, h0, t0, u, v, w, cos_t, ds, inv_bc;
    double photons;  // FP64: the longitudinal profile sums it
    float sb1x, sb1y, sb1z, sb2x, sb2y, sb2z;
    int32_t boff;   // first bunch of the step inside the tile
    int32_t sidx;   // index of the step inside the tile
    uint32_t ctr1;  // counter word 1 of the step's random numbers
    int32_t pad;
};
static_assert(sizeof(StepEntry<1>) == 128, "step entry size");

template <>
struct alignas(16) StepEntry<0> {
    double x0, y0, h0, t0, u, v, w, cos_t, ds, inv_bc;
    double sb1x, sb1y, sb1z, sb2x, sb2y, sb2z, photons;
    int32_t boff;
    int32_t sidx;
};
static_assert(sizeof(StepEntry<0>) == 144, "step entry size");

// per-wave counters kept in LDS (wave-uniform increments by lane 0)
enum WaveCounter { kWcBunches = 0, kWcEmitting, kWcHits, kWcDrop0, kWcCount = kWcDrop0 + CKV_N_DROP };

// Without the profile the whole table is staged in LDS.  With it, only the
// lowest kLdsTableEntries entries (nodes for FP64, cells for mixed, i.e. up to
// 76.8 km above the observation level on a 50 m grid) are, to leave room for
// the per-wave histograms; lookups above them read the same entries from HBM.
constexpr int kLdsTableEntries = 1536;

__host__ __device__ inline int lds_entries(int prec, int n_nodes, bool prof)
{
    const int n = prec == 0 ? n_nodes : n_nodes - 1;
    return prof && n > kLdsTableEntries ? kLdsTableEntries : n;
}

__host__ __device__ inline size_t table_bytes(int prec, int n_nodes, bool prof)
{
    return (size_t)lds_entries(prec, n_nodes, prof) *
           (prec == 0 ? kNode64 * sizeof(double) : kCell32 * sizeof(float));
}

__host__ __device__ inline size_t wave_bytes(int prec, int tile_segs, int n_tel, int prof_bins)
{
    size_t b = (size_t)tile_segs * (prec == 0 ? sizeof(StepEntry<0>) : sizeof(StepEntry<1>));
    b += kWave * sizeof(int32_t);                       // flag row
    if (prec == 0) b += (size_t)tile_segs * sizeof(uint32_t);   // counter words (FP64 path)
    b += (size_t)kWcCount * sizeof(int64_t);            // counters
    b += ((size_t)n_tel * sizeof(int32_t) + 15) & ~(size_t)15;   // telescope counters
    b += (size_t)prof_bins * (sizeof(double) + sizeof(uint32_t));  // profile of the tile
    return (b + 15) & ~(size_t)15;
}

constexpr int kSoftIdBits = 24;                          // bunch index bits of a list id
constexpr unsigned long long kSoftListInvalid = 1ull << 62;   // or-ed into the count

// Screening pass: the candidate bunches of ballot words bits[0..nw-1] (bit b of
// word q: bunch j0 + 64 q + b of the tile) go to the list.  One atomic claims exactly
// their slots; lane q writes the ids of word q, the step of its first bunch found
// by binary search over the tile's stash (first-bunch offsets ascend) and the
// later ones by moving forward from there (the lanes' searches overlap; this
// measured faster than word-by-word writes with consecutive slots).  lst (its
// offset in the dynamic LDS, as for bits and stash) holds
// {tile's first step, ids, capacity, count, tile's emitting steps}.  Called by
// the whole wave.
template <typename E>
__device__ __noinline__ void soft_list_flush(uint32_t lst_at, uint32_t bits_at, uint32_t stash_at, int64_t j0,
                                             int nw, int lane)
{
    // the wave's areas, by their offsets in the dynamic LDS (LDS accesses, not
    // generic ones)
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t* lst = reinterpret_cast<const int64_t*>(lds + lst_at);
    const uint64_t* bits = reinterpret_cast<const uint64_t*>(lds + bits_at);
    const E* stash = reinterpret_cast<const E*>(lds + stash_at);
    // (the caller's lane 0 wrote lst before the call; the wave's LDS accesses are in order)
    const int64_t l_g0 = lst[0], l_ids = lst[1], l_cap = lst[2], l_count = lst[3], l_emit = lst[4];
    uint64_t word = lane < nw ? bits[lane] : 0ull;
    const int c = __popcll(word);
    const int64_t incl = wave_incl_scan((int64_t)c);
    const int64_t tot = wave_last(incl);
    if (tot == 0) return;
    using GU64 = __attribute__((address_space(1))) unsigned long long;
    unsigned long long* count = (unsigned long long*)reinterpret_cast<GU64*>(l_count);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)tot);
    base = __shfl(base, 0);
    const int64_t g0 = l_g0, cap = l_cap;
    uint64_t* ids = (uint64_t*)reinterpret_cast<GU64*>(l_ids);
    int64_t slot = (int64_t)base + (incl - c);
    if (!word) return;
    const int n_emit = (int)l_emit;
    const int32_t jw = (int32_t)(j0 + kWave * lane);     // bunch of bit 0
    int32_t jj = jw + __builtin_ctzll(word);
    int lo = 0, hi = n_emit;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (stash[mid].boff <= jj) lo = mid; else hi = mid;
    }
    int32_t boff = stash[lo].boff;
    int32_t next = lo + 1 < n_emit ? stash[lo + 1].boff : INT_MAX;
    uint64_t step = (uint64_t)(g0 + stash[lo].sidx);
    for (;;) {
        while (jj >= next) {
            ++lo;
            boff = next;
            next = lo + 1 < n_emit ? stash[lo + 1].boff : INT_MAX;
            step = (uint64_t)(g0 + stash[lo].sidx);
        }
        const int32_t k = jj - boff;
        if ((uint32_t)k >= (1u << kSoftIdBits) || step >= (1ull << (64 - kSoftIdBits)))
            atomicOr(count, kSoftListInvalid);
        else if (slot < cap)
            ids[slot] = (step << kSoftIdBits) | (uint64_t)(uint32_t)k;
        ++slot;
        word &= word - 1;
        if (!word) break;
        jj = jw + __builtin_ctzll(word);
    }
}

// --------------------------------------------------------------------------
// the bunch kernel
// --------------------------------------------------------------------------
// FEAT bits: kFeatProfile (longitudinal profile), kFeatExact (grazing bunches
// traced exactly); each combination is its own kernel, so runs without them
// carry none of their code or registers.
constexpr int kFeatProfile = 1;
constexpr int kFeatExact = 2;
constexpr int kFeatSearch = 4;   // node tables: binary search per bunch (alone, 32-step tiles)
constexpr int kFeatCurved = 8;   // spherical shells, every bunch traced exactly (alone, 32-step tiles)
constexpr int kFeatWide = 16;    // mixed kernel built for <= 8 waves per workgroup (twice the registers)
// soft-response screening (mixed, alone, 32-step tiles): bunch counts frozen, each
// bunch tested against spheres of the soft cut radius plus a margin, the candidates'
// ids listed; no records
constexpr int kFeatScreen = 32;
// FP64 kernel built for 16 waves per workgroup (128 registers, four waves per SIMD):
// only the lowest kLdsTableEntries nodes of the table fit the LDS beside 16 wave
// areas, the rare lookups above them read HBM (alone, no other feature)
constexpr int kFeatNarrow = 64;
// per wave, after the regular area: list state {tile's first step, ids, capacity,
// count, emitting steps, unused} and the ballot words of the candidate bunches
constexpr int kScreenWords = 64;
constexpr size_t kScreenWaveBytes = (6 + kScreenWords) * sizeof(int64_t);

__host__ __device__ inline size_t search_bytes(int n_nodes)
{
    return ((size_t)(2 * n_nodes - 1) * sizeof(double) + 15) & ~(size_t)15;
}

// LDS layout of the bunch kernel: the atmosphere table (whole or in part), the node
// altitudes of the search variant, then the sphere table {X, Y, R^2}
template <int PREC, int FEAT>
__device__ __forceinline__ size_t tel_lds_offset(const Args& a)
{
    constexpr bool PARTIAL = (FEAT & (kFeatProfile | kFeatScreen | kFeatNarrow)) != 0;
    constexpr bool SEARCH = (FEAT & kFeatSearch) != 0;
    return ((table_bytes(PREC, a.n_nodes, PARTIAL) + 15) & ~(size_t)15) + (SEARCH ? search_bytes(a.n_nodes) : 0);
}

// sphere table in LDS: {X, Y, R^2} per sphere (at most CKV_MAX_TEL: 24 KB)
__host__ __device__ inline size_t tel_bytes(int n_tel)
{
    return ((size_t)n_tel * 3 * sizeof(double) + 15) & ~(size_t)15;
}

// Workgroup size the variant is compiled for: the FP64 kernel and the exact-path
// variants (grazing, curved) carry FP64 tracing state and get the registers of
// 8 waves; the mixed kernel is built for 16 waves (128 registers, the most
// waves per SIMD) and, as the wide variant, for up to 8 (256 registers: no
// spills, faster where step setup weighs more than bunches, e.g. at large
// zenith angles); the launch's wave count picks the build.
constexpr int emit_threads(int prec, int feat)
{
    return (feat & kFeatNarrow) ? 1024
           : (prec == 0 || (feat & (kFeatExact | kFeatCurved | kFeatWide)) != 0) ? 512 : 1024;
}

// Screening cull (soft response, plane-parallel atmosphere, FP64 pass as computed by
// soft_bunch).  A step's bunches leave from E(s) = P0 + s a, s in [0, L], in directions
// p = cos_t a + sin_t e with e a unit vector normal to a.  With T(d) = d_h / w_d
// (horizontal part over downward cosine) a bunch reaches the ground at
// g = E_h + T(p) S, where S = int T4(x) dh over the path, T4 the four-term series of
// (1 + x)^(-1/2) and x = q (psi - psi_e), q = 1 / (n_e w_p)^2 (App. B, the horizontal
// displacement, here as the moment series).  All of E(s) project along a to one point
// G = P0_h + (h0 - h_obs) T(a), so g - G = dh (T(p) - T(a)) - T(p) (dh - S), and:
// |T(p) - T(a)| = sin_t |(e x a)_h| / (w_p w_a), with |(e x a)_h| in [w_a, 1];
// w_p lies in [cos(zeta_a + t), cos(zeta_a - t)]; for x in [0, 1] (psi non-increasing
// with altitude) 0 <= 1 - T4(x) <= x/2, for |x| <= 1/2 |1 - T4(x)| <= 4|x|/5; and
// x <= x0 / w_p^2.  The bunch weights a sphere of radius R centred at c on the ground
// only if its observed line passes within R of c, so only if |g - c| <= R / w_o, with
// w_o^2 >= 1 - rho2 (1 - w_p^2).  Hence a step whose sphere centres all lie outside
// the annulus returned here (centre G, |d^2 - mid| <= half) gives no bunch a soft
// weight.  The bound takes a margin of 0.1 m plus 1e-6 relative for rounding; it is
// not applied (false) where its conditions fail: a direction not unit to 1e-9, w_a
// below 0.05, x0 / w_p^2 above 1/2 or w_o near zero.
__device__ inline bool screen_annulus(const Args& a, double x0, double y0, double h0, double u,
                                      double v, double w, double len, double ct, double st,
                                      double& gx, double& gy, double& mid, double& half)
{
    const double n2 = u * u + v * v + w * w;
    if (!(fabs(n2 - 1.0) <= 1e-9) || !(w >= 0.05)) return false;
    const double sa = sqrt(fmax(0.0, (1.0 - w) * (1.0 + w)));
    const double s_hi = st * (1.0 + 1e-9) + 1e-12, s_lo = fmax(st * (1.0 - 1e-9) - 1e-12, 0.0);
    // w_p of the bunches the FP64 pass keeps (w_p > w_min)
    const double wp_hi = fmin(1.0, w * ct + sa * s_hi + 1e-12);
    const double wp_lo = fmax(w * ct - sa * s_hi - 1e-12, a.w_min);
    if (!(wp_lo > 0.0)) return false;
    const double iw2 = 1.0 / (wp_lo * wp_lo);
    if (!(a.cull_x0 * iw2 <= 0.5)) return false;
    const double B = a.cull_b0 * iw2;                          // bound of |1 - S / dh|
    const double t_max = sqrt((1.0 - wp_lo) * (1.0 + wp_lo)) / wp_lo;   // bound of |T(p)|
    const double dh0 = h0 - a.h_obs;
    const double dh_top = fmax(dh0, 0.0), dh_bot = fmax(dh0 - len * w, 0.0);
    const double f_lo = s_lo / wp_hi - B * t_max;
    const double f_hi = s_hi / (wp_lo * w) + B * t_max;
    const double r_lo = f_lo > 0.0 ? dh_bot * f_lo : 0.0;      // |g - G| in [r_lo, r_hi]
    const double r_hi = dh_top * f_hi;
    const double wo2 = 1.0 - fmin(1.0, a.cull_rho2 * (1.0 - wp_lo) * (1.0 + wp_lo));
    if (!(wo2 > 1e-6)) return false;
    const double reach = a.cull_rmax / sqrt(wo2);
    const double m = 0.1 + 1e-6 * (dh_top + r_hi);
    const double inner = fmax(r_lo - reach - m, 0.0), outer = r_hi + reach + m;
    const double iw = 1.0 / w;
    gx = x0 + dh0 * (u * iw);
    gy = y0 + dh0 * (v * iw);
    mid = 0.5 * (outer * outer + inner * inner);
    half = 0.5 * (outer * outer - inner * inner) * (1.0 + 1e-9) + 1e-6;
    return true;
}

// The sphere test of the cull for a tile of at most 32 steps, step l in lane l: lanes
// l and l + 32 test the lower half [0, nh) and the upper half [n_tel - nh, n_tel) of
// the sphere table (STRIDE doubles per sphere, X and Y first; one sphere twice when
// n_tel is odd), the same count and stride in both, in a uniform loop whose loads do
// not wait on the tests before them.  ok: the lane's step has an annulus (gx, gy, mid,
// half from screen_annulus).  True in lane l < 32 when step l's annulus holds a sphere
// centre.  Called by the whole wave.
template <int STRIDE>
__device__ __forceinline__ bool annulus_holds_centre(const double* tel, int n_tel, int lane, int ok, double gx,
                                                     double gy, double mid, double half)
{
    const int src = lane & (kWave / 2 - 1);
    const int ok_s = __shfl(ok, src);
    gx = __shfl(gx, src);
    gy = __shfl(gy, src);
    mid = __shfl(mid, src);
    half = __shfl(half, src);
    const int nh = (n_tel + 1) >> 1;
    const double* tp = tel + STRIDE * (lane < kWave / 2 ? 0 : n_tel - nh);
    bool reach = false;
#pragma unroll 4
    for (int i = 0; i < nh; ++i) {
        const double dx = tp[STRIDE * i] - gx, dy = tp[STRIDE * i + 1] - gy;
        reach |= fabs(fma(dy, dy, dx * dx) - mid) <= half;
    }
    reach = reach && ok_s;
    const uint64_t rm = __ballot(reach);
    return (((rm >> src) | (rm >> (src + kWave / 2))) & 1ull) != 0;
}

// Step setups of a tile, one per lane (emitting steps compacted into the stash),
// the bunch-count scan and the step-level counters; returns the tile's bunch
// count and this lane's step state.  Not inlined: the step arrays' pointers and
// the setup's registers then take no room in the bunch loop.  Called by the
// whole wave.
struct TileSetup {
    int64_t total;
    int excl;
    bool emits;
};

template <int PREC, int TS, int FEAT>
__device__ __forceinline__ TileSetup tile_setup(const Args& a, int64_t g0, int nseg, int64_t seg_id0,
                                                int lane, uint64_t lt_mask, StepEntry<PREC>* stash,
                                                uint32_t* sctr, int64_t* wcnt, int64_t* lst)
{
    constexpr bool SCREEN = (FEAT & kFeatScreen) != 0;
    using T = typename std::conditional<PREC == 0, double, float>::type;
    using Entry = StepEntry<PREC>;
    int64_t nb = 0;
    int status = -2;   // -2: no step in this lane
    Setup st;
    double len = 0.0;
    if (lane < nseg) {
        // screening: the frozen count and the length loaded with the step's inputs,
        // not after them
        const int64_t f = SCREEN ? a.nb_frozen[g0 + lane] : 0;
        if (SCREEN) len = a.len[g0 + lane];
        step_setup(a, g0 + lane, st);
        status = st.status;
        if (st.status < 0) nb = st.nb;
        if (SCREEN && st.status < 0) {
            // the soft response's sub-steps: the frozen count, light or not at
            // the current atmosphere decided above
            if (f > 0) {
                nb = f;
                st.ds = len / (double)f;
            } else {
                nb = 0;
                status = -4;
            }
        }
    }
    // the tile-size limit on the frozen counts, before the screening cull
    const int64_t nb_all = nb;
    if constexpr (SCREEN) {
        static_assert(TS <= kWave / 2, "the cull splits the spheres between half-waves");
        extern __shared__ __align__(16) unsigned char lds[];
        const double* tel_sh = reinterpret_cast<const double*>(lds + tel_lds_offset<PREC, FEAT>(a));
        // steps whose bunches can weight no sphere are not screened (screen_annulus)
        double cgx = 0.0, cgy = 0.0, cmid = 0.0, chalf = -1.0;
        int ok = 0;
        if (lane < nseg && status == -1 && a.cull_rmax > 0.0)
            ok = screen_annulus(a, st.x0, st.y0, st.h0, st.u, st.v, st.w, len, st.cos_t, st.sin_t, cgx, cgy,
                                cmid, chalf) ? 1 : 0;
        const bool reached = annulus_holds_centre<3>(tel_sh, a.n_tel, lane, ok, cgx, cgy, cmid, chalf);
        if (ok && !reached) {
            nb = 0;
            status = -4;
        }
    }
    int64_t incl = PREC == 1 ? wave_incl_scan_shfl(nb) : wave_incl_scan(nb);
    int64_t total = scalar64(wave_last(incl));
    const int64_t total_all =
        SCREEN ? scalar64(wave_last(PREC == 1 ? wave_incl_scan_shfl(nb_all) : wave_incl_scan(nb_all))) : total;
    if (total_all >= ((int64_t)1 << 30)) {
        // bunch offsets inside a tile are 32-bit: refuse such a tile
        if (lane == 0 && a.result) atomicOr(&a.result->error, 2);
        total = 0;
        incl = 0;
        nb = 0;
        status = status == -1 ? -3 : status;
    }
    const bool emits = status == -1;
    const uint64_t emit_mask = __ballot(emits);
    if (SCREEN && lane == 0) {
        lst[0] = g0;
        lst[4] = __popcll(emit_mask);
    }
    const int excl = (int)(incl - nb);      // first bunch of this lane's step
    if (emits) {
        Entry& e = stash[__popcll(emit_mask & lt_mask)];
        const int64_t g = g0 + lane;
        const uint32_t ctr1 = a.step_id ? a.step_id[g] : (uint32_t)(seg_id0 + lane);
        if constexpr (PREC == 1) e.ctr1 = ctr1;
        else sctr[lane] = ctr1;
        if constexpr (PREC == 1 && (FEAT & kFeatProfile) == 0) {
            // the called setup keeps the inputs it loaded rather than a second round
            // (the profile build, short of registers, measured faster reloading)
            e.x0 = st.x0;
            e.y0 = st.y0;
            e.h0 = st.h0;
            e.t0 = st.t0;
            e.u = st.u;
            e.v = st.v;
            e.w = st.w;
        } else {
            e.x0 = a.x0[g];
            e.y0 = a.y0[g];
            e.h0 = a.h0[g];
            e.t0 = a.t0[g];
            e.u = a.u[g];
            e.v = a.v[g];
            e.w = a.w[g];
        }
        e.cos_t = st.cos_t;
        e.ds = st.ds;
        e.inv_bc = st.inv_bc;
        e.sb1x = (T)(st.sin_t * st.b1x);
        e.sb1y = (T)(st.sin_t * st.b1y);
        e.sb1z = (T)(st.sin_t * st.b1z);
        e.sb2x = (T)(st.sin_t * st.b2x);
        e.sb2y = (T)(st.sin_t * st.b2y);
        e.sb2z = (T)(st.sin_t * st.b2z);
        e.photons = st.photons;
        e.boff = excl;
        e.sidx = lane;
    }
    {
        const int d_mass = __popcll(__ballot(status == CKV_DROP_MASS));
        const int d_thr = __popcll(__ballot(status == CKV_DROP_THRESHOLD));
        const int d_nf = __popcll(__ballot(status == CKV_DROP_NONFINITE));
        if (lane == 0) {
            wcnt[kWcBunches] += total;
            wcnt[kWcEmitting] += __popcll(emit_mask);
            wcnt[kWcDrop0 + CKV_DROP_MASS] += d_mass;
            wcnt[kWcDrop0 + CKV_DROP_THRESHOLD] += d_thr;
            wcnt[kWcDrop0 + CKV_DROP_NONFINITE] += d_nf;
        }
    }
    return TileSetup{total, (int)(incl - nb), status == -1};
}

// The same as a called function (the mixed kernel's choice: its step setup's
// registers and the step arrays' pointers then take no room in the bunch loop,
// 100 -> 8 scalar spills; the FP64 kernel, with 256 registers, runs faster inline).
template <int PREC, int TS, int FEAT>
__device__ __noinline__ TileSetup tile_setup_call(uint64_t args_at, int64_t g0, int nseg, int64_t seg_id0,
                                                  int lane, uint64_t lt_mask, uint32_t stash_at,
                                                  uint32_t sctr_at, uint32_t wcnt_at, uint32_t lst_at)
{
    extern __shared__ __align__(16) unsigned char lds[];
    // the launch's argument block, at the address the kernel passes: wave-uniform and
    // read-only, so the setup reads it with scalar loads
    const uint64_t at_u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(args_at >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)args_at);
    const Args& a = *(const Args*)reinterpret_cast<const __attribute__((address_space(4))) Args*>(at_u);
    return tile_setup<PREC, TS, FEAT>(a, g0, nseg, seg_id0, lane, lt_mask,
                                      reinterpret_cast<StepEntry<PREC>*>(lds + stash_at),
                                      reinterpret_cast<uint32_t*>(lds + sctr_at),
                                      reinterpret_cast<int64_t*>(lds + wcnt_at),
                                      reinterpret_cast<int64_t*>(lds + lst_at));
}

template <int PREC, int TS, int FEAT>
__global__ void __launch_bounds__(emit_threads(PREC, FEAT)) emit_kernel(Args a)
{
    constexpr bool PROF = (FEAT & kFeatProfile) != 0;
    constexpr bool EXACT = (FEAT & kFeatExact) != 0;
    constexpr bool SEARCH = (FEAT & kFeatSearch) != 0;
    constexpr bool CURVED = (FEAT & kFeatCurved) != 0;
    constexpr bool SCREEN = (FEAT & kFeatScreen) != 0;
    constexpr bool NARROW = (FEAT & kFeatNarrow) != 0;
    constexpr bool PARTIAL = PROF || SCREEN || NARROW;   // table staged in part, the rest from HBM
    constexpr bool SLOWPATH = EXACT || CURVED;    // lanes that leave the moment series
    using T = typename std::conditional<PREC == 0, double, float>::type;
    using Entry = StepEntry<PREC>;
    extern __shared__ __align__(16) unsigned char lds[];

    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;

    // ---- stage the atmosphere table once per workgroup
    const size_t tab_bytes = table_bytes(PREC, a.n_nodes, PARTIAL);
    {
        const uint4* src = reinterpret_cast<const uint4*>(PREC == 0 ? (const void*)a.node64
                                                                    : (const void*)a.cell32);
        uint4* dst = reinterpret_cast<uint4*>(lds);
        const int n16 = (int)(tab_bytes / 16);
        for (int q = threadIdx.x; q < n16; q += blockDim.x) dst[q] = src[q];
    }
    // node tables: altitudes and inverse widths after the table
    double* hn_lds = reinterpret_cast<double*>(lds + ((tab_bytes + 15) & ~(size_t)15));
    const size_t srch_bytes = SEARCH ? search_bytes(a.n_nodes) : 0;
    if (SEARCH)
        for (int q = threadIdx.x; q < 2 * a.n_nodes - 1; q += blockDim.x) hn_lds[q] = a.hnodes[q];
    // sphere table {X, Y, R^2} after them
    double* tel_sh = reinterpret_cast<double*>(lds + tel_lds_offset<PREC, FEAT>(a));
    for (int q = threadIdx.x; q < a.n_tel; q += blockDim.x) {
        tel_sh[3 * q] = a.tel[4 * q];
        tel_sh[3 * q + 1] = a.tel[4 * q + 1];
        tel_sh[3 * q + 2] = a.tel[4 * q + 3];
    }
    const size_t wv_bytes = wave_bytes(PREC, TS, a.n_tel, PROF ? a.prof_bins : 0);
    unsigned char* wbase = lds + ((tab_bytes + 15) & ~(size_t)15) + srch_bytes + tel_bytes(a.n_tel) +
                           (size_t)wave * (wv_bytes + (SCREEN ? kScreenWaveBytes : 0));
    // screening: list state and ballot words after the wave's regular area
    int64_t* lst = reinterpret_cast<int64_t*>(wbase + wv_bytes);
    uint64_t* bits = reinterpret_cast<uint64_t*>(lst + 6);
    if (SCREEN && lane == 0) {
        lst[1] = (int64_t)a.list_ids;
        lst[2] = a.list_cap;
        lst[3] = (int64_t)a.list_count;
    }
    Entry* stash = reinterpret_cast<Entry*>(wbase);
    int32_t* flags = reinterpret_cast<int32_t*>(wbase + TS * sizeof(Entry));
    // FP64 path: counter word per step (the mixed path keeps it in its step record)
    uint32_t* sctr = reinterpret_cast<uint32_t*>(flags + kWave);
    int64_t* wcnt = reinterpret_cast<int64_t*>(sctr + (PREC == 0 ? ((TS + 1) & ~1) : 0));
    int32_t* tcount = reinterpret_cast<int32_t*>(wcnt + kWcCount);
    // profile of the current tile: photons (FP64) and bunches per depth bin
    double* hph = reinterpret_cast<double*>(
        reinterpret_cast<unsigned char*>(tcount) + (((size_t)a.n_tel * sizeof(int32_t) + 15) & ~(size_t)15));
    uint32_t* hbu = reinterpret_cast<uint32_t*>(hph + a.prof_bins);
    for (int k = lane; k < a.n_tel; k += kWave) tcount[k] = 0;
    if (PROF)
        for (int k = lane; k < a.prof_bins; k += kWave) { hph[k] = 0.0; hbu[k] = 0u; }
    if (lane < kWcCount) wcnt[lane] = 0;
    flags[lane] = 0;
    __syncthreads();

    const double* tab64 = reinterpret_cast<const double*>(lds);
    const float* tab32 = reinterpret_cast<const float*>(lds);
    const T a1 = (T)-0.5, a2 = (T)0.375, a3 = (T)-0.3125, a4 = (T)0.2734375;
    const double inv_c = 1.0 / kSpeedOfLight;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t le_mask = lt_mask | (1ull << lane);
    const float step32 = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, (float)a.step)));
    // n - 1 at the observation level, for the observed direction
    const double inv_nobs64 = 1.0 / a.n_obs;
    const float d_obs = (float)(a.n_obs - 1.0);
    const float inv_1pdobs = 1.0f / (1.0f + d_obs);
    // grazing limit of the drop rules, read once (a scalar load in the bunch loop made
    // its wait cover the loop's LDS reads as well).  Screening keeps bunches down to
    // w_min - 1e-6, ten times the mixed direction's error: the FP64 candidate pass
    // applies the exact rule.
    const double w_graze = __builtin_bit_cast(double, scalar64(__builtin_bit_cast(int64_t,
                               SCREEN ? a.w_min - 1e-6 : a.w_min)));

    int64_t blk = -1;          // current staging block; -1: none yet, -2: staging full
    int blk_fill = 0;
    bool lost = false;         // a crossing of this wave found no slot (tile marked)
    int64_t rblk = -1;         // current run block; -1: none yet
    int rfill = 0;
    const int64_t n_tiles = a.ctrl[kNumTiles];

    // Atmosphere at an emission point in cell ci at fraction f (node tables: dcell_
    // above the cell's lower node h_i): psi_e and D_k = int_{h_obs}^{h_e} (psi -
    // psi_e)^k dh, k = 1..5.  Below h_i the node moments are shifted to psi_e,
    // sum_j C(k,j) (-psi_e)^(k-j) P_j(h_i) with P_0(h_i) = h_i - h_obs (Pascal-triangle
    // shift); inside the cell psi is linear from psi_i to psi_e, so the rest is
    // dz (psi_i - psi_e)^k / (k+1).  The bunch loop takes D_1..D_4 for the advance;
    // the arrival time, needed only for a crossing's record, takes D_5 as well.
    struct CellMoments { T psi_e, D1, D2, D3, D4, D5; };
    auto cell_moments = [&](int ci, T f, double dcell_) {
        T psi_i, dpsi, P0, P1, P2, P3, P4, P5;
        // LDS read always (index clamped into the staged part); the rare
        // lookups above it are replaced by a read from HBM.  The FP32 table's two
        // reads go through their own address spaces, so the compiler cannot fuse
        // them into one generic (flat) load for every lookup.  The FP64 narrow build
        // keeps the fused generic load: typed, it spills more and runs 0.5 %
        // slower.
        if (PREC == 0) {
            double n0[6], n1;
            {
                const int cl = PARTIAL ? min(ci, a.lds_entries - 2) : ci;
                const double* nd = tab64 + (size_t)kNode64 * cl;
                for (int q = 0; q < 6; ++q) n0[q] = nd[q];
                n1 = nd[kNode64];
            }
            if (PARTIAL && ci + 1 >= a.lds_entries) {
                const double* nd = a.node64 + (size_t)kNode64 * ci;
                for (int q = 0; q < 6; ++q) n0[q] = __builtin_nontemporal_load(nd + q);
                n1 = __builtin_nontemporal_load(nd + kNode64);
            }
            psi_i = n0[0];
            dpsi = n1 - n0[0];
            P0 = SEARCH ? hn_lds[ci] - a.h_obs : (double)ci * a.step;
            P1 = n0[1]; P2 = n0[2]; P3 = n0[3]; P4 = n0[4]; P5 = n0[5];
        } else {
            f32x4 c_a, c_b;
            {
                const int cl = PARTIAL ? min(ci, a.lds_entries - 1) : ci;
                const LdsF32x4* cc = as_lds4(tab32 + (size_t)kCell32 * cl);
                c_a = cc[0];
                c_b = cc[1];
            }
            if (PARTIAL && ci >= a.lds_entries) {
                const HbmF32x4* cg = as_hbm4(a.cell32 + (size_t)kCell32 * ci);
                c_a = cg[0];
                c_b = cg[1];
            }
            psi_i = c_a.x; dpsi = c_a.y; P1 = c_a.z; P2 = c_a.w;
            P3 = c_b.x; P4 = c_b.y; P5 = c_b.z;
            P0 = c_b.w;
        }
        CellMoments m;
        m.psi_e = psi_i + f * dpsi;
        const T dz = SEARCH ? (T)dcell_ : f * (PREC == 0 ? (T)a.step : (T)step32);
        const T c1 = -m.psi_e;
        T X0 = P0, X1 = P1, X2 = P2, X3 = P3, X4 = P4, X5 = P5;
        X5 += c1 * X4; X4 += c1 * X3; X3 += c1 * X2; X2 += c1 * X1; X1 += c1 * X0;
        X5 += c1 * X4; X4 += c1 * X3; X3 += c1 * X2; X2 += c1 * X1;
        X5 += c1 * X4; X4 += c1 * X3; X3 += c1 * X2;
        X5 += c1 * X4; X4 += c1 * X3;
        X5 += c1 * X4;
        const T del = -f * dpsi;               // psi_i - psi_e
        const T e1 = dz * del, e2 = e1 * del, e3 = e2 * del, e4 = e3 * del, e5 = e4 * del;
        m.D1 = X1 + e1 * (T)0.5;
        m.D2 = X2 + e2 * (T)(1.0 / 3.0);
        m.D3 = X3 + e3 * (T)0.25;
        m.D4 = X4 + e4 * (T)0.2;
        m.D5 = X5 + e5 * (T)(1.0 / 6.0);
        return m;
    };
    // Index terms at emission (n_e = 1 + delta_e) for a photon of vertical cosine w:
    // n_e, 1/w, n_e / n_obs (the observed direction's scale), q = 1/(n_e w)^2, 1/n_e
    // and n_e^2.
    struct IndexTerms { double ne, inv_w; T ratio, q, inv_ne, ne2; };
    auto index_terms = [&](T psi_e, double pw) {
        IndexTerms x;
        x.ne2 = (T)1 + psi_e;
        if (PREC == 0) {
            x.ne = sqrt(1.0 + (double)psi_e);
            x.ratio = (T)(x.ne * inv_nobs64);
            x.inv_w = rcp64(pw);
            x.inv_ne = (T)rcp64(x.ne);
            x.q = (T)(x.inv_w * x.inv_w) * (x.inv_ne * x.inv_ne);
        } else {
            const float de = (float)psi_e * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_sqrtf(1.0f + (float)psi_e));
            x.ne = 1.0 + (double)de;
            x.ratio = 1.0f + (de - d_obs) * inv_1pdobs;
            // reciprocal of w: the hardware estimate (relative error below 2^-24 on
            // this chip) and one Newton step, 2e-15 relative
            const double r_w = __builtin_amdgcn_rcp(pw);
            x.inv_w = fma(r_w, fma(-pw, r_w, 1.0), r_w);
            x.q = (T)__builtin_amdgcn_rcpf((float)x.ne2 * (float)(pw * pw));
            x.inv_ne = (T)__builtin_amdgcn_rcpf(1.0f + de);
        }
        return x;
    };
    // series part of the horizontal advance, S - dh = sum_{k>=1} a_k q^k D_k
    auto advance_series = [&](const CellMoments& m, T q) {
        return q * (a1 * m.D1 + q * (a2 * m.D2 + q * (a3 * m.D3 + q * a4 * m.D4)));
    };
    // travel time from the emission height dh above the observation level:
    // c * time * w = n_e dh + (1/n_e) [D1 + sum_{k>=1} a_k q^k (n_e^2 D_k + D_{k+1})]
    //              = n_e dh + (1/n_e) [D1 + n_e^2 s_corr + sum_{k>=1} a_k q^k D_{k+1}]
    auto travel_time = [&](const CellMoments& m, const IndexTerms& ix, T s_corr, double dh) {
        const T q = ix.q;
        const T t_corr = m.D1 + ix.ne2 * s_corr +
                         q * (a1 * m.D2 + q * (a2 * m.D3 + q * (a3 * m.D4 + q * a4 * m.D5)));
        const double ctw = fma(ix.ne, dh, (double)(t_corr * ix.inv_ne));
        return ctw * ix.inv_w * inv_c;
    };

    // tiles are claimed from the counter.  The mixed kernel takes each wave's first
    // tile by its index in the grid and offsets later claims by the grid's wave count,
    // so the launch does not start with every wave's atomic on the one counter (the
    // FP64 kernel measured slower with it: the extra scalar state spills)
    constexpr bool kStaticFirst = PREC == 1;
    const int64_t n_waves_grid = kStaticFirst ? (int64_t)gridDim.x * (blockDim.x / kWave) : 0;
    const int64_t t_first = kStaticFirst ? scalar64((int64_t)blockIdx.x * (blockDim.x / kWave) + wave) : 0;
    bool first_tile = kStaticFirst;
    for (;;) {
        int64_t t = t_first;
        if (!first_tile) {
            if (lane == 0)
                t = n_waves_grid +
                    (int64_t)atomicAdd((unsigned long long*)&a.ctrl[SCREEN ? kScreenCounter : kTileCounter], 1ull);
            t = kStaticFirst ? scalar64(t) : uniform(t);
        }
        first_tile = false;
        if (t >= n_tiles) break;
        // shower of the tile
        int lo = 0, hi = a.n_showers;   // tiles_before[lo] <= t < tiles_before[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.tiles_before[mid] <= t) lo = mid; else hi = mid;
        }
        const int s = lo;
        const int64_t g0 = a.shower_first[s] + (t - a.tiles_before[s]) * (int64_t)TS;
        const int64_t gend = min(g0 + (int64_t)TS, a.seg_offsets[s + 1]);
        const int nseg = (int)(gend - g0);
        const uint32_t shower_id = a.shower_ids ? a.shower_ids[s] : (uint32_t)s;
        const int64_t seg_id0 = (a.seg_id_base ? a.seg_id_base[s] : 0) + (g0 - a.seg_offsets[s]);
        const double t_ref = a.t_ref[s];
        int32_t thits = 0;         // crossings of this tile (wave-uniform)

        // ---- step setups, one per lane; emitting steps are compacted.  The mixed
        // kernel calls it out of line, handing the callee the arguments where the
        // launch put them (the kernel argument segment) rather than a private copy.
        TileSetup ts_;
        if constexpr (PREC == 1) {
            auto at = [&](const void* p) { return (uint32_t)((const unsigned char*)p - lds); };
            const uint64_t args_at = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
            ts_ = tile_setup_call<PREC, TS, FEAT>(args_at, g0, nseg, seg_id0, lane, lt_mask, at(stash), at(sctr),
                                                  at(wcnt), at(lst));
        } else {
            ts_ = tile_setup<PREC, TS, FEAT>(a, g0, nseg, seg_id0, lane, lt_mask, stash, sctr, wcnt, lst);
        }
        const int64_t total = ts_.total;
        const bool emits = ts_.emits;
        const int excl = ts_.excl;
        wave_lds_sync();

        // ---- bunches of the tile, one per lane
        for (int64_t c0 = 0; c0 < total; c0 += kWave) {
            const int32_t j = (int32_t)(c0 + lane);
            const bool active = j < total;
            // step of bunch j: emitting steps starting at or before c0, plus the
            // steps starting inside this chunk at or before j (flag row)
            const int cnt0 = __popcll(__ballot(emits && excl <= (int)c0));
            if (emits && excl > (int)c0 && excl < (int)c0 + kWave) flags[excl - (int)c0] = 1;
            wave_lds_sync();
            const uint64_t starts = __ballot(flags[lane] != 0);
            flags[lane] = 0;
            const int si = cnt0 - 1 + __popcll(starts & le_mask);
            // Philox round keys, advanced on the scalar unit inside the loop
            const uint32_t opaque = (uint32_t)(c0 >> 40);   // 0; keeps the schedule in the loop
            uint32_t kr0 = a.key0 + opaque, kr1 = a.key1 + opaque;

            bool alive = false;
            int drop_why = -1;
            // read only in lanes that emit a live bunch: left undefined elsewhere
            double xg, yg, he;
            int32_t k, sidx;
            double uod, vod;   // observed direction for the sphere test (live bunches)
            int pbin = -1;     // depth bin of the bunch for the profile, -1: not counted
            bool screen_all = false;   // screening: listed whatever its sphere tests say
            double fcell, dcell = 0.0;   // fraction and height of the emission point in its cell
            int ci;
            // what a crossing's record needs beyond the above; the record itself is
            // completed only in chunks that hold a crossing
            double t_rec;        // mixed fast path: emission time - t_ref; else the arrival time
            double w_rec;        // mixed fast path: w of the photon at emission
            T f_rec;             // mixed fast path: fraction of the emission point in its cell
            bool fast_rec = false;
            uint32_t r2_rec;     // the wavelength's draw
            if (active) {
                const Entry& e = stash[si];
                k = j - e.boff;
                sidx = e.sidx;
                // Philox4x32-10 with counter (k, step index in shower, shower id, 0)
                uint32_t c_0 = (uint32_t)k, c_2 = shower_id, c_3 = 0u;
                uint32_t c_1;
                if constexpr (PREC == 1) c_1 = e.ctr1;
                else c_1 = sctr[sidx];
#pragma unroll
                for (int rr = 0; rr < 10; ++rr) {
                    const uint64_t p0 = (uint64_t)0xD2511F53u * c_0;
                    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c_2;
                    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c_1, kr0, 0x96);
                    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c_3, kr1, 0x96);
                    c_1 = (uint32_t)p1;
                    c_3 = (uint32_t)p0;
                    c_0 = n0;
                    c_2 = n2;
                    kr0 += 0x9E3779B9u;
                    kr1 += 0xBB67AE85u;
                }
                const uint32_t r0 = c_0, r1 = c_1, r2 = c_2;
                // emission point, uniform inside sub-step k (FP64)
                const double u0 = fma((double)r0, 2.3283064365386963e-10, 1.1641532182693481e-10);
                const double s_along = ((double)k + u0) * e.ds;
                const double tu = e.u, tv = e.v, tw = e.w;
                double xe, ye, ze;
                {
                    // rounded as the FP64 definition rounds it: the drop tests and the
                    // profile bin take their decisions on this value (and, curved, on
                    // the altitude of (x, y, z))
#pragma clang fp contract(off)
                    he = e.h0 - s_along * tw;
                    if (CURVED) {
                        xe = e.x0 + s_along * tu;
                        ye = e.y0 + s_along * tv;
                    }
                }
                if (!CURVED) {
                    xe = fma(s_along, tu, e.x0);
                    ye = fma(s_along, tv, e.y0);
                }
                ze = he;
                if (CURVED) he = curved_altitude(a.earth_r, xe, ye, ze);
                const double te = fma(s_along, e.inv_bc, e.t0);
                // table cell and fraction of the emission altitude (index and depth)
                if (SEARCH) {
                    // node tables: branch-free binary search in LDS (sec. 3.3.1)
                    int lo = 0;
                    for (int stp = a.search_pow2; stp > 0; stp >>= 1) {
                        const int c = lo + stp;
                        if (c < a.n_nodes - 1 && hn_lds[c] <= he) lo = c;
                    }
                    ci = lo;
                    dcell = he - hn_lds[ci];
                    fcell = dcell * hn_lds[a.n_nodes + ci];
                } else {
                    const double xcell = (he - a.h_obs) * a.inv_step;
                    ci = min((int)xcell, a.n_nodes - 2);
                    fcell = xcell - (double)ci;
                }
                if (PROF && he >= a.h_obs && he < a.h_top) pbin = profile_bin(a, ci, fcell);
                const double ct = e.cos_t;
                // direction on the Cherenkov cone
                double pu, pv, pw;
                if (PREC == 0) {
                    double sp, cp;
                    sincos_turns64(r1, sp, cp);
                    pu = ct * tu + (cp * (double)e.sb1x + sp * (double)e.sb2x);
                    pv = ct * tv + (cp * (double)e.sb1y + sp * (double)e.sb2y);
                    pw = ct * tw - (cp * (double)e.sb1z + sp * (double)e.sb2z);
                } else {
                    float sp, cp;
                    sincos_turns_hw(r1, sp, cp);
                    const float px = fmaf(cp, (float)e.sb1x, sp * (float)e.sb2x);
                    const float py = fmaf(cp, (float)e.sb1y, sp * (float)e.sb2y);
                    const float pz = fmaf(cp, (float)e.sb1z, sp * (float)e.sb2z);
                    pu = fma(ct, tu, (double)px);
                    pv = fma(ct, tv, (double)py);
                    pw = fma(ct, tw, -(double)pz);
                }
                r2_rec = r2;
                // drop rules, in this order: below the observation level, above the top,
                // upward, grazing (selects, no branches)
                const bool d_below = he < a.h_obs, d_above = he >= a.h_top;
                const bool d_up = !CURVED && pw <= 0.0, d_graze = !CURVED && pw <= w_graze;
                const bool kept = !d_below && !d_above && !d_up;
                drop_why = d_below ? CKV_DROP_BELOW_OBS
                           : d_above ? CKV_DROP_ABOVE_TOP
                           : d_up ? CKV_DROP_UPWARD
                           : (d_graze && !EXACT) ? CKV_DROP_GRAZING : -1;
                // slow: traced exactly, cell by cell (grazing bunches; every bunch when curved,
                // whose upward and turning drops the tracer decides)
                bool slow = kept && (CURVED || (EXACT && d_graze));
                if (SLOWPATH && slow) {
                    alive = true;
                    if (PREC == 1) {
                        // a grazing ray magnifies a direction error by 1/w^2 on the
                        // ground: redo the direction in FP64 (frame of the step, FP64
                        // azimuth), as the FP64 path has it
                        const double Dz = -tw, sgn = copysign(1.0, Dz);
                        const double ia = -1.0 / (sgn + Dz), ib = tu * tv * ia;
                        const double b1x = 1.0 + sgn * tu * tu * ia, b1y = sgn * ib, b1z = -sgn * tu;
                        const double b2x = ib, b2y = sgn + tv * tv * ia, b2z = -tv;
                        const double st_ = sqrt((1.0 - ct) * (1.0 + ct));
                        double sp, cp;
                        sincos_turns64(r1, sp, cp);
                        pu = ct * tu + st_ * (cp * b1x + sp * b2x);
                        pv = ct * tv + st_ * (cp * b1y + sp * b2y);
                        pw = ct * tw - st_ * (cp * b1z + sp * b2z);
                    }
                    double T_x = 0.0;
                    if (CURVED) {
                        const int stc = propagate_curved(a, xe, ye, ze, he, pu, pv, pw, xg, yg, T_x,
                                                         uod, vod);
                        if (stc >= 0) {
                            drop_why = stc;
                            alive = false;
                        }
                    } else {
                        double ne_x;
                        propagate_exact(a, xe, ye, he, pu, pv, pw, xg, yg, T_x, ne_x);
                        uod = pu * ne_x / a.n_obs;
                        vod = pv * ne_x / a.n_obs;
                    }
                    t_rec = (te - t_ref) + T_x;
                }
                if (drop_why < 0 && !slow) {
                    alive = true;
                    // ---- atmosphere at the emission altitude (uniform table, no search)
                    const T f = (T)fcell;
                    const CellMoments m = cell_moments(ci, f, dcell);
                    const IndexTerms ix = index_terms(m.psi_e, pw);
                    // horizontal advance: S = dh + sum_{k>=1} a_k q^k D_k
                    const double dh = he - a.h_obs;
                    const T s_corr = advance_series(m, ix.q);
                    const double S = dh + (double)s_corr;
                    const double adv = ix.inv_w * S;
                    if (SCREEN) {
                        // bound of this path's ground-point error (direction error of the
                        // FP32 cone vector through 1/w and u/w^2, FP32 series corrections
                        // through q ~ 1/w^2 and 1/w): where it passes half the screening
                        // margin the sphere test cannot be trusted and the bunch is listed
                        const double e_g = dh * ix.inv_w * (kScreenErrDir * (1.0 + ix.inv_w) +
                                                            kScreenErrSeries * ix.inv_w * ix.inv_w);
                        screen_all = e_g > 0.5 * kScreenMargin;
                    }
                    xg = fma(pu, adv, xe);
                    yg = fma(pv, adv, ye);
                    // the sphere test takes the observed direction at the path's
                    // precision (FP64 path: before the record's FP32 rounding)
                    const T uT = (T)pu * ix.ratio, vT = (T)pv * ix.ratio;
                    uod = (double)uT;
                    vod = (double)vT;
                    if constexpr (PREC == 0) {
                        // FP64: the arrival time at once (keeping the inputs of its
                        // recomputation live costs this build more than it saves)
                        t_rec = (te - t_ref) + travel_time(m, ix, s_corr, dh);
                    } else {
                        t_rec = te - t_ref;
                        w_rec = pw;
                        f_rec = f;
                        fast_rec = true;
                    }
                }
            }
            {
                const int d0 = __popcll(__ballot(drop_why == CKV_DROP_BELOW_OBS));
                const int d1 = __popcll(__ballot(drop_why == CKV_DROP_ABOVE_TOP));
                const int d2 = __popcll(__ballot(drop_why == CKV_DROP_UPWARD));
                const int d3 = __popcll(__ballot(drop_why == CKV_DROP_GRAZING));
                if (lane == 0 && (d0 | d1 | d2 | d3)) {
                    wcnt[kWcDrop0 + CKV_DROP_BELOW_OBS] += d0;
                    wcnt[kWcDrop0 + CKV_DROP_ABOVE_TOP] += d1;
                    wcnt[kWcDrop0 + CKV_DROP_UPWARD] += d2;
                    wcnt[kWcDrop0 + CKV_DROP_GRAZING] += d3;
                }
            }
            if (PROF) {
                // runs of lanes with the same step and bin (bunches of a step are
                // consecutive lanes and their depth is monotonic in k): the first lane
                // of each run adds the whole run, so LDS atomics do not collide
                const bool member = pbin >= 0;
                const int key = member ? (si << 8) | pbin : -1;     // pbin < 256
                // the previous lane's key (DPP wave shift right by one; lane 0 gets -2)
                const int key_prev = __builtin_amdgcn_update_dpp(-2, key, 0x138, 0xf, 0xf, false);
                const bool head = member && key_prev != key;
                const uint64_t mem_mask = __ballot(member), head_mask = __ballot(head);
                if (head) {
                    const uint64_t after = lane == kWave - 1 ? 0ull : (~0ull << (lane + 1));
                    const uint64_t ends = (~mem_mask | head_mask) & after;
                    const int len = (ends ? __builtin_ctzll(ends) : kWave) - lane;
                    atomicAdd(&hph[pbin], (double)len * stash[si].photons);
                    atomicAdd(&hbu[pbin], (uint32_t)len);
                }
            }
            // ---- candidate spheres (ascending telescope index)
            int cur = 0, cend = 0;
            int first = -1;          // the cell's first sphere, known without a list read
            bool brute = false;
            if (alive) {
                const double wo2 = 1.0 - uod * uod - vod * vod;
                if (wo2 >= kLevelW2[0]) {
                    const double fx = (xg - a.gx0) * a.inv_cell, fy = (yg - a.gy0) * a.inv_cell;
                    if (fx >= 0.0 && fy >= 0.0 && fx < (double)a.nx && fy < (double)a.ny) {
                        const int cidx = grid_level(wo2) * a.level_cells + (int)fx * a.ny + (int)fy;
                        const uint2 ce = a.cell_ent[cidx];
                        cur = (int)ce.x;
                        cend = cur + (int)(ce.y & 0xFFFFu);
                        first = (int)(ce.y >> 16);
                    }
                } else {
                    brute = true;
                    cend = a.n_tel;
                }
            }
            int my_next = INT_MAX;
            auto advance = [&]() {
                my_next = INT_MAX;
                while (cur < cend) {
                    const int kt = brute ? cur : (first >= 0 ? first : (int)a.cell_list[cur]);
                    first = -1;
                    ++cur;
                    const double* tq = tel_sh + 3 * kt;     // sphere table in LDS
                    const double tX = tq[0], tY = tq[1], tR2 = tq[2];
                    const double dx = xg - tX, dy = yg - tY;
                    const double b = dx * uod + dy * vod;
                    const double disc = b * b - (dx * dx + dy * dy - tR2);
                    if (disc >= 0.0) { my_next = kt; break; }
                }
            };
            advance();
            if constexpr (SCREEN) {
                // candidates of the soft response: one ballot word per 64 bunches,
                // flushed to the list when the buffer is full and at the tile's end
                const uint64_t m = __ballot(my_next != INT_MAX || screen_all);
                const int w = (int)((c0 >> 6) & (kScreenWords - 1));
                if (lane == 0) bits[w] = m;
                if (w == kScreenWords - 1 || c0 + kWave >= total) {
                    wave_lds_sync();
                    soft_list_flush<Entry>((uint32_t)((unsigned char*)lst - lds), (uint32_t)((unsigned char*)bits - lds),
                                           (uint32_t)((unsigned char*)stash - lds), c0 - (int64_t)w * kWave, w + 1,
                                           lane);
                }
            } else {
                // ---- the records of the crossing bunches.  About one chunk in five holds
                // a crossing, so the wavelength and the record's roundings are done here,
                // for those lanes; the mixed path also takes the arrival time's series
                // (the only user of D_5 and 1/n_e) here, recomputed from the table rather
                // than kept live through the sphere tests.
                float uo, vo, t_f, he_f, photons, lam;
                int32_t k_rec, sidx_rec;
                if (__ballot(my_next != INT_MAX)) {
                    if (my_next != INT_MAX) {
                        const Entry& er = stash[si];
                        k_rec = j - er.boff;
                        sidx_rec = er.sidx;
                        photons = (float)er.photons;
                        if (PREC == 0) {
                            lam = (float)rcp64(a.inv_l1 - fma((double)r2_rec, 2.3283064365386963e-10,
                                                              1.1641532182693481e-10) * a.dl);
                        } else {
                            const float u2 = fmaf((float)r2_rec, 2.3283064365386963e-10f,
                                                  1.16415321826934814e-10f);
                            lam = __builtin_amdgcn_rcpf(fmaf(-u2, (float)a.dl, (float)a.inv_l1));
                        }
                        double tarr = t_rec;
                        if constexpr (PREC == 1) {
                            if (fast_rec) {
                                const CellMoments m = cell_moments(ci, f_rec, dcell);
                                const IndexTerms ix = index_terms(m.psi_e, w_rec);
                                tarr += travel_time(m, ix, advance_series(m, ix.q), he - a.h_obs);
                            }
                        }
                        uo = (float)uod;
                        vo = (float)vod;
                        t_f = (float)tarr;
                        he_f = (float)he;
                    }
                }
                // ---- record crossings; telescopes in ascending order, lanes (bunches) in order
                while (__ballot(my_next != INT_MAX)) {
                    const int kmin = wave_min_sparse(my_next, INT_MAX);
                    const bool mine = my_next == kmin;
                    const uint64_t mask = __ballot(mine);
                    const int nmine = __popcll(mask);
                    const int below = __popcll(mask & lt_mask);
                    const int rank0 = tcount[kmin];
                    thits += nmine;
                    // staging slots: the first `room` crossings fill the current
                    // block, the rest start a newly claimed one
                    const int room = blk >= 0 ? kStageBlock - blk_fill : 0;
                    int64_t nbk = -2;
                    if (nmine > room && blk != -2) {
                        if (blk >= 0 && lane == 0) a.stage_fill[blk] = kStageBlock;
                        if (lane == 0) nbk = (int64_t)atomicAdd((unsigned long long*)&a.ctrl[kBlockCounter], 1ull);
                        nbk = uniform(nbk);
                        if (nbk >= a.stage_blocks) nbk = -2;
                    }
                    if (nmine > room && nbk < 0 && !lost) {
                        // crossings of this tile find no slot: the run's written prefix
                        // ends before it (this wave's later tiles come after it)
                        lost = true;
                        if (lane == 0) atomicMin((unsigned long long*)&a.ctrl[kFirstLost], (unsigned long long)t);
                    }
                    if (mine) {
                        int64_t slot = -1;
                        if (below < room) slot = blk * kStageBlock + blk_fill + below;
                        else if (nbk >= 0) slot = nbk * kStageBlock + (below - room);
                        if (slot >= 0) {
                            StageEntry* se = a.stage + slot;
                            const double* tp = a.tel + 4 * kmin;
                            float4* ef = reinterpret_cast<float4*>(se);
                            ef[0] = make_float4((float)(xg - tp[0]), (float)(yg - tp[1]), uo, vo);
                            ef[1] = make_float4(t_f, he_f, photons, lam);
                            uint4* eu = reinterpret_cast<uint4*>(se);
                            eu[2] = make_uint4((uint32_t)t, (uint32_t)kmin | ((uint32_t)sidx_rec << 16),
                                               (uint32_t)(rank0 + below), (uint32_t)k_rec);
                        }
                    }
                    if (nmine > room) {
                        if (blk != -2) {
                            blk = nbk;               // -2 when the staging area is full
                            blk_fill = nmine - room;
                        }
                    } else {
                        blk_fill += nmine;
                    }
                    if (lane == 0) tcount[kmin] = rank0 + nmine;
                    wave_lds_sync();
                    if (mine) advance();
                }
            }
        }
        // ---- per-telescope crossings of this tile as runs (ascending telescope)
        wave_lds_sync();
        if (!SCREEN && t < a.max_tiles) {
            int nz = 0;
            for (int k0 = 0; k0 < a.n_tel; k0 += kWave) {
                const int kk = k0 + lane;
                nz += __popcll(__ballot(kk < a.n_tel && tcount[kk] != 0));
            }
            // run slots from the wave's current block of kRunBlock (a tile with more
            // runs than a block takes enough whole blocks of its own)
            int64_t base = 0;
            if (nz > 0) {
                if (rblk < 0 || rfill + nz > kRunBlock) {
                    const int nblk = (nz + kRunBlock - 1) / kRunBlock;
                    int64_t b = 0;
                    if (lane == 0) b = (int64_t)atomicAdd((unsigned long long*)&a.ctrl[kRunCounter],
                                                          (unsigned long long)nblk);
                    rblk = scalar64(uniform(b));
                    rfill = 0;
                }
                base = rblk * kRunBlock + rfill;
                rfill = nz > kRunBlock ? kRunBlock : rfill + nz;
            }
            const bool fits = base + nz <= a.run_cap;
            if (!fits && !lost) {
                lost = true;
                if (lane == 0) atomicMin((unsigned long long*)&a.ctrl[kFirstLost], (unsigned long long)t);
            }
            int done = 0;
            for (int k0 = 0; k0 < a.n_tel; k0 += kWave) {
                const int kk = k0 + lane;
                const int32_t c = kk < a.n_tel ? tcount[kk] : 0;
                const uint64_t m = __ballot(c != 0);
                if (c != 0) {
                    if (fits)
                        a.runs[base + done + __popcll(m & lt_mask)] = ((int64_t)kk << kRunTelShift) | c;
                    tcount[kk] = 0;
                }
                done += __popcll(m);
            }
            if (lane == 0) {
                a.tile_run_off[t] = base;
                a.tile_run_n[t] = fits ? nz : 0;
                a.tile_hits[t] = thits;
            }
            if (lane == 0) wcnt[kWcHits] += thits;
        }
        // ---- profile of this tile into its shower's row
        for (int kk = lane; PROF && kk < a.prof_bins; kk += kWave) {
            const uint32_t c = hbu[kk];
            if (c) {
                const int64_t g = (int64_t)s * a.prof_bins + kk;
                atomicAdd(&a.prof_ph[g], hph[kk]);
                atomicAdd((unsigned long long*)&a.prof_bu[g], (unsigned long long)c);
                hph[kk] = 0.0;
                hbu[kk] = 0u;
            }
        }
        wave_lds_sync();
    }

    // ---- close the staging block and publish counters: the workgroup's waves are
    // summed in LDS and the first wave adds the sums, one atomic per counter and
    // workgroup (one per wave queued thousands of atomics on the counters' line at
    // the end of every launch)
    if (blk >= 0 && lane == 0) a.stage_fill[blk] = blk_fill;
    __syncthreads();
    if (wave == 0 && lane < kWcCount) {
        const size_t wstride = wv_bytes + (SCREEN ? kScreenWaveBytes : 0);
        const unsigned char* w0 = reinterpret_cast<const unsigned char*>(wcnt);
        int64_t v = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w)
            v += reinterpret_cast<const int64_t*>(w0 + (size_t)w * wstride)[lane];
        const int slot = lane == kWcBunches ? kBunches
                       : lane == kWcEmitting ? kEmitting
                       : lane == kWcHits ? kHits
                       : kDrop0 + (lane - kWcDrop0);
        if (v) atomicAdd((unsigned long long*)&a.ctrl[slot], (unsigned long long)v);
    }
}

// --------------------------------------------------------------------------
// init: control block, shower validation, tile and row-block counts
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) init_kernel(Args a)
{
    __shared__ int64_t sh_t[1024], sh_b[1024];
    __shared__ int err;
    for (int q = threadIdx.x; q < kCtrlSlots; q += blockDim.x) a.ctrl[q] = 0;
    if (threadIdx.x == 0) err = 0;
    __syncthreads();
    const int64_t TS = a.tile_segs;
    int64_t run_t = 0, run_b = 0;
    for (int base = 0; base < a.n_showers; base += blockDim.x) {
        const int s = base + threadIdx.x;
        int64_t nt = 0, nbk = 0;
        if (s < a.n_showers) {
            const int64_t lo = a.seg_offsets[s], hi = a.seg_offsets[s + 1];
            if (lo < 0 || hi < lo || hi > a.n || (s == 0 && lo != 0) ||
                (s == a.n_showers - 1 && hi != a.n))
                err = 1;
            // the run starts at the cursor: showers before its shower have no tiles,
            // its shower starts at the cursor's step
            int64_t first = lo;
            if (s < a.cur_shower) {
                first = hi;
            } else if (s == a.cur_shower) {
                if (a.cur_step < lo || a.cur_step > hi) err = 1;
                first = a.cur_step < lo ? lo : (a.cur_step > hi ? hi : a.cur_step);
            }
            if (a.shower_first) a.shower_first[s] = first;
            const int64_t cnt = hi >= first ? hi - first : 0;
            nt = (cnt + TS - 1) / TS;
            nbk = (nt + kRowBlock - 1) / kRowBlock;
        }
        sh_t[threadIdx.x] = nt;
        sh_b[threadIdx.x] = nbk;
        __syncthreads();
        for (int d = 1; d < (int)blockDim.x; d <<= 1) {
            int64_t xt = 0, xb = 0;
            if ((int)threadIdx.x >= d) { xt = sh_t[threadIdx.x - d]; xb = sh_b[threadIdx.x - d]; }
            __syncthreads();
            sh_t[threadIdx.x] += xt;
            sh_b[threadIdx.x] += xb;
            __syncthreads();
        }
        if (s < a.n_showers) {
            a.tiles_before[s] = run_t + sh_t[threadIdx.x] - nt;
            a.blocks_before[s] = run_b + sh_b[threadIdx.x] - nbk;
        }
        run_t += sh_t[blockDim.x - 1];
        run_b += sh_b[blockDim.x - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.tiles_before[a.n_showers] = run_t;
        a.blocks_before[a.n_showers] = run_b;
        if (run_t > a.max_tiles || run_b > a.max_row_blocks) err = 1;
        a.ctrl[kNumTiles] = err ? 0 : run_t;
        a.ctrl[kNumRowBlocks] = err ? 0 : run_b;
        a.ctrl[kFirstLost] = err ? 0 : run_t;      // no lost tile yet
        if (a.result) {
            // the bunch path's finalize fills the rest; the soft entry points report
            // the error word only
            ckv_result* r = a.result;
            r->n_bunches = r->n_hits = r->n_records = r->n_emitting = r->n_tiles = 0;
            for (int d = 0; d < CKV_N_DROP; ++d) r->drops[d] = 0;
            r->resume_step = a.n;
            r->resume_shower = a.n_showers;
            r->overflow = 0;
            r->error = err;
            r->reserved = 0;
        }
    }
}

// --------------------------------------------------------------------------
// finalize
// --------------------------------------------------------------------------
__device__ __forceinline__ int find_shower(const int64_t* before, int n_showers, int64_t x)
{
    int lo = 0, hi = n_showers;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (before[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Row block b of shower s holds the shower's tiles [t0, t1) below; blocks and tiles
// are both numbered shower by shower, so block order is tile order.
__device__ __forceinline__ void block_tiles(const Args& a, int64_t b, int& s, int64_t& t0, int64_t& t1)
{
    s = find_shower(a.blocks_before, a.n_showers, b);
    t0 = a.tiles_before[s] + (b - a.blocks_before[s]) * kRowBlock;
    t1 = min(t0 + (int64_t)kRowBlock, a.tiles_before[s + 1]);
}

// Tile of the j-th run (0 <= q < the lanes' total) among lanes 0..m-1 holding
// inclusive run counts `incl` (one tile per lane): the first lane whose count
// passes q.  m is a power of two, the same in every lane.
__device__ __forceinline__ int run_tile(int64_t incl, int64_t q, int m)
{
    int lo = 0;
    for (int step = m >> 1; step > 0; step >>= 1)
        if (__shfl(incl, lo + step - 1) <= q) lo += step;
    return lo;
}

// Adds the runs of tiles [t0, t1) into acc[telescope] (LDS) with the whole
// workgroup.  Each wave takes groups of kRowBlock / waves tiles: its lanes load
// the group's run counts and offsets in one round, then walk the group's runs in
// flat order (a run per lane), so the loads of different tiles are not chained.
__device__ __forceinline__ void add_runs(const Args& a, int64_t t0, int64_t t1, int32_t* acc)
{
    const int lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    int g = kRowBlock / nw;                         // tiles per group: a power of two
    if (g < 1) g = 1;
    for (int64_t base = t0 + (int64_t)wave * g; base < t1; base += (int64_t)nw * g) {
        const int64_t t = base + lane;
        const bool mine = lane < g && t < t1;
        const int n = mine ? a.tile_run_n[t] : 0;
        const int64_t off = mine ? a.tile_run_off[t] : 0;
        const int64_t incl = wave_incl_scan((int64_t)n);
        const int64_t total = wave_last(incl);
        // the whole wave runs every round (the shuffles read every lane)
        for (int64_t q0 = 0; q0 < total; q0 += kWave) {
            const int64_t q = q0 + lane;
            const int j = run_tile(incl, q, g);
            const int64_t off_j = __shfl(off, j), first_j = __shfl(incl, j) - __shfl((int64_t)n, j);
            if (q < total) {
                const int64_t r = a.runs[off_j + (q - first_j)];
                atomicAdd(&acc[(int)(r >> kRunTelShift)], (int32_t)(r & kRunValueMask));
            }
        }
    }
}

// A: per row block: crossings per telescope (block_sums, telescope-major:
// block_sums[k * max_row_blocks + b]) and in all (block_hits).
__global__ void __launch_bounds__(256) block_sum_kernel(Args a)
{
    extern __shared__ int32_t acc[];               // n_tel
    __shared__ unsigned long long tot;
    const int64_t nblk = a.ctrl[kNumRowBlocks];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        for (int k = threadIdx.x; k < a.n_tel; k += blockDim.x) acc[k] = 0;
        if (threadIdx.x == 0) tot = 0;
        __syncthreads();
        int s;
        int64_t t0, t1;
        block_tiles(a, b, s, t0, t1);
        add_runs(a, t0, t1, acc);
        for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x)
            atomicAdd(&tot, (unsigned long long)a.tile_hits[t]);
        __syncthreads();
        for (int k = threadIdx.x; k < a.n_tel; k += blockDim.x)
            a.block_sums[(int64_t)k * a.max_row_blocks + b] = acc[k];
        if (threadIdx.x == 0) a.block_hits[b] = (int64_t)tot;
        __syncthreads();
    }
}

// B: the written prefix.  Without a lost tile and with every crossing within the
// capacity it is the whole run.  Otherwise it ends at the first tile that is
// lost or whose crossings would pass the capacity; the row block holding that
// tile gets its sums again over the tiles before it.  One workgroup.
__global__ void __launch_bounds__(1024) cutoff_kernel(Args a)
{
    extern __shared__ int32_t acc[];               // n_tel
    __shared__ int64_t part[1024];
    __shared__ int first_thread;
    __shared__ int64_t cut_tile, cut_block, cut_records, blk_b, blk_before;
    const int64_t n_tiles = a.ctrl[kNumTiles], nblk = a.ctrl[kNumRowBlocks];
    const int64_t lost = a.ctrl[kFirstLost];
    const int64_t hits = a.ctrl[kHits];
    if (lost >= n_tiles && hits <= a.capacity) {
        if (threadIdx.x == 0) {
            a.ctrl[kCutTile] = n_tiles;
            a.ctrl[kCutBlocks] = nblk;
            a.ctrl[kRecords] = hits;
        }
        return;
    }
    // the row block holding the lost tile bounds the search
    int64_t b_lim = nblk;
    if (lost < n_tiles) {
        const int sl = find_shower(a.tiles_before, a.n_showers, lost);
        b_lim = a.blocks_before[sl] + (lost - a.tiles_before[sl]) / kRowBlock + 1;
    }
    // first block whose crossings, added to those before it, pass the capacity
    const int nt = blockDim.x;
    const int64_t chunk = (b_lim + nt - 1) / nt;
    const int64_t lo = (int64_t)threadIdx.x * chunk, hi = min(lo + chunk, b_lim);
    int64_t mine = 0;
    for (int64_t b = lo; b < hi; ++b) mine += a.block_hits[b];
    part[threadIdx.x] = mine;
    if (threadIdx.x == 0) first_thread = nt;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {
        const int64_t y = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    const int64_t before = part[threadIdx.x] - mine;
    if (lo < hi && part[threadIdx.x] > a.capacity) atomicMin(&first_thread, (int)threadIdx.x);
    __syncthreads();
    if ((int)threadIdx.x == (first_thread < nt ? first_thread : nt - 1)) {
        // walk this thread's blocks to the first that passes (the lost tile's block
        // when none does)
        int64_t cum = first_thread < nt ? before : part[nt - 1] - a.block_hits[b_lim - 1];
        int64_t b = first_thread < nt ? lo : b_lim - 1;
        if (first_thread < nt)
            while (b + 1 < hi && cum + a.block_hits[b] <= a.capacity) cum += a.block_hits[b++];
        blk_b = b;
        blk_before = cum;
    }
    __syncthreads();
    // the tile: first of block blk_b that is lost or passes the capacity
    if (threadIdx.x == 0) {
        int s;
        int64_t t0, t1;
        block_tiles(a, blk_b, s, t0, t1);
        int64_t cum = blk_before, t = t0;
        while (t < t1 && t < lost && cum + a.tile_hits[t] <= a.capacity) cum += a.tile_hits[t++];
        cut_tile = t;
        cut_block = t > t0 ? blk_b + 1 : blk_b;
        cut_records = cum;
    }
    __syncthreads();
    // sums of the boundary block over its tiles before the cut
    const int64_t b = blk_b;
    int s;
    int64_t t0, t1;
    block_tiles(a, b, s, t0, t1);
    for (int k = threadIdx.x; k < a.n_tel; k += blockDim.x) acc[k] = 0;
    __syncthreads();
    add_runs(a, t0, min(t1, cut_tile), acc);
    __syncthreads();
    for (int k = threadIdx.x; k < a.n_tel; k += blockDim.x)
        a.block_sums[(int64_t)k * a.max_row_blocks + b] = acc[k];
    if (threadIdx.x == 0) {
        a.ctrl[kCutTile] = cut_tile;
        a.ctrl[kCutBlocks] = cut_block;
        a.ctrl[kRecords] = cut_records;
    }
}

// C: per (shower, telescope), one wave: exclusive scan over the shower's row
// blocks below the cut, 8 x 64 blocks per round
__global__ void __launch_bounds__(256) rowblock_scan_kernel(Args a)
{
    const int lane = lane_id();
    const int64_t nst = (int64_t)a.n_showers * a.n_tel;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const bool have_tiles = a.ctrl[kNumTiles] > 0;
    const int64_t cutb = a.ctrl[kCutBlocks];
    for (int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; q < nst;
         q += waves) {
        const int s = (int)(q / a.n_tel), k = (int)(q % a.n_tel);
        int64_t run = 0;
        if (have_tiles) {
            int32_t* col = a.block_sums + (int64_t)k * a.max_row_blocks;
            const int64_t b_end = min(a.blocks_before[s + 1], cutb);
            // the loads issue before the first store and one wave scan of the lane
            // sums serves all
            constexpr int G = 8;
            for (int64_t b0 = a.blocks_before[s]; b0 < b_end; b0 += G * kWave) {
                const int64_t bl = b0 + (int64_t)G * lane;
                int32_t x[G];
                int64_t lsum = 0;
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    x[j] = bl + j < b_end ? col[bl + j] : 0;
                    lsum += x[j];
                }
                const int64_t incl = wave_incl_scan(lsum);
                int64_t pre = run + incl - lsum;
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    if (bl + j < b_end) col[bl + j] = (int32_t)pre;
                    pre += x[j];
                }
                run += wave_last(incl);
            }
        }
        if (lane == 0) a.shower_tel[q] = (int32_t)run;
    }
}

// D: per row block below the cut, one wave: each run's count becomes the
// crossings of its (shower, telescope) in earlier tiles.  The block's runs are
// gathered into LDS when they fit (one load round per tile list), walked tile by
// tile there, and written back.
constexpr int kPrefixLdsRuns = 4096;

__global__ void __launch_bounds__(64) tile_prefix_kernel(Args a)
{
    extern __shared__ int32_t ctr[];               // n_tel counters, then the run buffer
    int64_t* buf = reinterpret_cast<int64_t*>(ctr + ((a.n_tel + 1) & ~1));
    const int lane = lane_id();
    const int64_t cutb = a.ctrl[kCutBlocks], cut = a.ctrl[kCutTile];
    for (int64_t b = blockIdx.x; b < cutb; b += gridDim.x) {
        int s;
        int64_t t0, t1;
        block_tiles(a, b, s, t0, t1);
        t1 = min(t1, cut);
        for (int k = lane; k < a.n_tel; k += kWave) ctr[k] = a.block_sums[(int64_t)k * a.max_row_blocks + b];
        // lane l: tile t0 + l (a block has at most 64 tiles)
        const int64_t tl = t0 + lane;
        const int n = tl < t1 ? a.tile_run_n[tl] : 0;
        const int64_t off = tl < t1 ? a.tile_run_off[tl] : 0;
        const int64_t incl = wave_incl_scan((int64_t)n);
        const int64_t total = wave_last(incl);
        const int my0 = (int)(incl - n);
        const bool in_lds = total <= kPrefixLdsRuns;
        // the block's runs into LDS in flat order, a run per lane (the loads of
        // different tiles are not chained)
        if (in_lds)
            for (int64_t q0 = 0; q0 < total; q0 += kWave) {
                const int64_t q = q0 + lane;
                const int j = run_tile(incl, q, kWave);
                const int64_t off_j = __shfl(off, j), first_j = __shfl(incl, j) - __shfl((int64_t)n, j);
                if (q < total) buf[q] = a.runs[off_j + (q - first_j)];
            }
        wave_lds_sync();
        for (int64_t t = t0; t < t1; ++t) {
            // the tile's count, offset and first slot from its lane (a uniform lane
            // index: a register read, not an LDS round trip)
            const int j = (int)(t - t0);
            const int nj = __builtin_amdgcn_readlane(n, j);
            const int64_t offj = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(off >> 32), j) << 32) |
                                           (uint32_t)__builtin_amdgcn_readlane((int)off, j));
            const int bj = __builtin_amdgcn_readlane(my0, j);
            for (int i = lane; i < nj; i += kWave) {
                const int64_t r = in_lds ? buf[bj + i] : a.runs[offj + i];
                const int tel = (int)(r >> kRunTelShift);
                const int32_t v = ctr[tel];
                const int64_t w = ((int64_t)tel << kRunTelShift) | v;
                if (in_lds) buf[bj + i] = w; else a.runs[offj + i] = w;
                ctr[tel] = v + (int32_t)(r & kRunValueMask);
            }
            wave_lds_sync();
        }
        if (in_lds)
            for (int64_t q0 = 0; q0 < total; q0 += kWave) {
                const int64_t q = q0 + lane;
                const int j = run_tile(incl, q, kWave);
                const int64_t off_j = __shfl(off, j), first_j = __shfl(incl, j) - __shfl((int64_t)n, j);
                if (q < total) a.runs[off_j + (q - first_j)] = buf[q];
            }
        wave_lds_sync();
    }
}

// D, for at most kPrefixDenseTel telescopes: per row block, one workgroup.  The
// block's runs go into a dense tiles x telescopes count matrix in LDS, each
// telescope's column is scanned from the crossings of earlier blocks, and each run
// takes its entry.  Nothing is serial over the block's tiles but one register sum
// per column, so the block costs a few memory round trips instead of a chain of
// LDS round trips per tile.
constexpr int kPrefixDenseTel = 128;

__global__ void __launch_bounds__(256) tile_prefix_dense_kernel(Args a)
{
    extern __shared__ int32_t mat[];               // kRowBlock x n_tel, row = tile
    __shared__ int64_t s_incl[kRowBlock], s_off[kRowBlock];
    const int tid = threadIdx.x, nt = a.n_tel;
    const int64_t cutb = a.ctrl[kCutBlocks], cut = a.ctrl[kCutTile];
    for (int64_t b = blockIdx.x; b < cutb; b += gridDim.x) {
        int s;
        int64_t t0, t1;
        block_tiles(a, b, s, t0, t1);
        t1 = min(t1, cut);
        const int ntl = (int)(t1 - t0);
        if (tid < kWave) {
            // lane l: tile t0 + l; inclusive run counts over the block's tiles
            const bool mine = tid < ntl;
            const int n = mine ? a.tile_run_n[t0 + tid] : 0;
            s_off[tid] = mine ? a.tile_run_off[t0 + tid] : 0;
            s_incl[tid] = wave_incl_scan((int64_t)n);
        }
        for (int q = tid; q < ntl * nt; q += blockDim.x) mat[q] = 0;
        __syncthreads();
        const int64_t total = s_incl[kRowBlock - 1];
        // the block's runs in flat order: run q's tile is the first whose inclusive
        // count passes q
        for (int64_t q = tid; q < total; q += blockDim.x) {
            int j = 0;
            for (int step = kRowBlock / 2; step > 0; step >>= 1)
                if (s_incl[j + step - 1] <= q) j += step;
            const int64_t first = j ? s_incl[j - 1] : 0;
            const int64_t r = a.runs[s_off[j] + (q - first)];
            mat[j * nt + (int)(r >> kRunTelShift)] = (int32_t)(r & kRunValueMask);
        }
        __syncthreads();
        // exclusive scan down each telescope's column
        for (int k = tid; k < nt; k += blockDim.x) {
            int32_t acc = a.block_sums[(int64_t)k * a.max_row_blocks + b];
            for (int j = 0; j < ntl; ++j) {
                const int32_t v = mat[j * nt + k];
                mat[j * nt + k] = acc;
                acc += v;
            }
        }
        __syncthreads();
        for (int64_t q = tid; q < total; q += blockDim.x) {
            int j = 0;
            for (int step = kRowBlock / 2; step > 0; step >>= 1)
                if (s_incl[j + step - 1] <= q) j += step;
            const int64_t first = j ? s_incl[j - 1] : 0;
            const int64_t g = s_off[j] + (q - first);
            const int tel = (int)(a.runs[g] >> kRunTelShift);
            a.runs[g] = ((int64_t)tel << kRunTelShift) | mat[j * nt + tel];
        }
        __syncthreads();
    }
}

// E: CSR offsets over (shower, telescope) and the run report
__global__ void __launch_bounds__(1024) csr_kernel(Args a)
{
    __shared__ int64_t sh[1024];
    const int64_t nst = (int64_t)a.n_showers * a.n_tel;
    int64_t run = 0;
    for (int64_t base = 0; base < nst; base += blockDim.x) {
        const int64_t q = base + threadIdx.x;
        const int64_t x = q < nst ? (int64_t)a.shower_tel[q] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int d = 1; d < (int)blockDim.x; d <<= 1) {
            int64_t y = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (q < nst) a.tel_offsets[q] = run + sh[threadIdx.x] - x;
        run += sh[blockDim.x - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.tel_offsets[nst] = run;
        ckv_result* r = a.result;
        const int64_t n_tiles = a.ctrl[kNumTiles], cut = a.ctrl[kCutTile];
        r->n_bunches = a.ctrl[kBunches];
        r->n_hits = a.ctrl[kHits];
        r->n_records = a.ctrl[kRecords];
        r->n_emitting = a.ctrl[kEmitting];
        r->n_tiles = n_tiles;
        for (int d = 0; d < CKV_N_DROP; ++d) r->drops[d] = a.ctrl[kDrop0 + d];
        if (cut < n_tiles) {
            const int sc = find_shower(a.tiles_before, a.n_showers, cut);
            r->resume_shower = sc;
            r->resume_step = a.shower_first[sc] + (cut - a.tiles_before[sc]) * (int64_t)a.tile_segs;
            r->overflow = 1;
        } else {
            r->resume_shower = a.n_showers;
            r->resume_step = a.n;
            r->overflow = 0;
        }
    }
}

// F: scatter the staged records of the written tiles to their final slots.  A
// slot's place is its (shower, telescope) offset, plus its telescope's crossings
// in earlier tiles of the shower (its run's value), plus its rank in the tile.
// Each thread takes kScatterSlots slots a round and issues the loads that do not
// depend on one another together: the block fills, then the entries (record and
// placement at once), then the tile's run list, the shower's offset and the
// shower (tile bounds staged in LDS for up to kScatterShowerLds showers), then the
// searches over the runs side by side.
constexpr int kScatterSlots = 2;
constexpr int kScatterShowerLds = 2048;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // plain 16-byte vector

struct ScatterSlot {
    u32x4 rec0, rec1, meta;
    int64_t off, base;
    int n, tel, shower, lo, len;
    bool live;
};

__device__ __forceinline__ void scatter_fill(const Args& a, ScatterSlot& x, int64_t q, int64_t nslots)
{
    const int64_t b = q < nslots ? q / kStageBlock : 0;
    x.live = q < nslots && (int)(q - b * kStageBlock) < a.stage_fill[b];
}

// (a slot that is not live reads slot 0, which every such slot shares)
__device__ __forceinline__ void scatter_entry(const Args& a, ScatterSlot& x, int64_t q)
{
    const u32x4* e = reinterpret_cast<const u32x4*>(a.stage + (x.live ? q : 0));
    x.rec0 = e[0];
    x.rec1 = e[1];
    x.meta = e[2];
}

__device__ __forceinline__ void scatter_tile(const Args& a, ScatterSlot& x, const int64_t* before, int64_t cut)
{
    const int64_t tile = x.meta.x;
    x.tel = (int)(x.meta.y & 0xFFFFu);
    x.live = x.live && tile < cut && x.tel < a.n_tel;
    x.n = 0;
    x.lo = 0;
    if (x.live) {
        x.shower = find_shower(before, a.n_showers, tile);
        x.off = a.tile_run_off[tile];
        x.n = a.tile_run_n[tile];
        x.base = a.tel_offsets[(int64_t)x.shower * a.n_tel + x.tel];
    }
    x.len = x.n;
}

// one halving step of the search for the tile's run of the slot's telescope (runs
// ascend by telescope)
__device__ __forceinline__ void scatter_halve(const Args& a, ScatterSlot& x)
{
    if (x.len > 1) {
        const int half = x.len >> 1;
        if ((int)(a.runs[x.off + x.lo + half] >> kRunTelShift) <= x.tel) x.lo += half;
        x.len -= half;
    }
}

__device__ __forceinline__ void scatter_store(const Args& a, const ScatterSlot& x, const int64_t* before)
{
    if (!x.live || x.n <= 0) return;
    const int64_t r = a.runs[x.off + x.lo];
    if ((int)(r >> kRunTelShift) != x.tel) return;
    const int64_t pos = x.base + (r & kRunValueMask) + x.meta.z;
    if (pos < 0 || pos >= a.capacity) return;
    u32x4* dst = reinterpret_cast<u32x4*>(a.records + 8 * pos);
    dst[0] = x.rec0;
    dst[1] = x.rec1;
    if (a.ids) {
        const int s = x.shower;
        a.ids[2 * pos] = a.shower_first[s] + ((int64_t)x.meta.x - before[s]) * (int64_t)a.tile_segs +
                         (int)(x.meta.y >> 16);
        a.ids[2 * pos + 1] = x.meta.w;
    }
}

__device__ __forceinline__ void scatter_pair(const Args& a, const int64_t* before, int64_t q0,
                                             int64_t stride, int64_t nslots, int64_t cut)
{
    ScatterSlot x, y;
    const int64_t q1 = q0 + stride;
    scatter_fill(a, x, q0, nslots);
    scatter_fill(a, y, q1, nslots);
    scatter_entry(a, x, q0);
    scatter_entry(a, y, q1);
    scatter_tile(a, x, before, cut);
    scatter_tile(a, y, before, cut);
    while (x.len > 1 || y.len > 1) {
        scatter_halve(a, x);
        scatter_halve(a, y);
    }
    scatter_store(a, x, before);
    scatter_store(a, y, before);
}

__global__ void __launch_bounds__(256) scatter_kernel(Args a)
{
    __shared__ int64_t s_before[kScatterShowerLds + 1];
    const bool lds_showers = a.n_showers <= kScatterShowerLds;
    if (lds_showers)
        for (int q = threadIdx.x; q <= a.n_showers; q += blockDim.x) s_before[q] = a.tiles_before[q];
    __syncthreads();
    const int64_t cut = a.ctrl[kCutTile];
    const int64_t nblk = min(a.ctrl[kBlockCounter], a.stage_blocks);
    const int64_t nslots = nblk * kStageBlock;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q0 < nslots; q0 += kScatterSlots * stride) {
        if (lds_showers) scatter_pair(a, s_before, q0, stride, nslots, cut);
        else scatter_pair(a, a.tiles_before, q0, stride, nslots, cut);
    }
}

// standalone bunch count per step (FP64, same operations as the bunch kernel)
__global__ void __launch_bounds__(256) count_kernel(Args a, int64_t* n_b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        Setup st;
        step_setup(a, i, st);
        n_b[i] = st.status >= 0 ? 0 : st.nb;
    }
}

// --------------------------------------------------------------------------
// Soft telescope response and its adjoint (differentiation pattern), FP64.
//   S_sk = sum photons * Phi(z),  A_sk = sum photons * Phi(z) * t,
//   z = (R^2 - rho^2) / (2 R sigma),
// with bunch counts frozen per step.  MODE 0 accumulates S and A; MODE 1
// recomputes every bunch from its random numbers and accumulates dL/dpsi_i and
// dL/dP_j(h_i) given dL/dS and dL/dA.
// --------------------------------------------------------------------------
struct SoftArgs {
    const int64_t* nb_frozen;
    double sigma;
    const double* gS;
    const double* gA;
    double* S;
    double* A;
    double* g_psi;
    double* g_P;
    double gx0, gy0, inv_cell;
    int32_t nx, ny, level_cells;
    const int32_t* cell_off;
    const uint16_t* cell_list;
    const uint2* cell_ent;      // per cell: {offset, count | first sphere << 16}
    // list of the bunches with a nonzero weight: written by the forward, read by the
    // adjoint (ids (step << kSoftIdBits) | k; count > capacity: incomplete)
    uint64_t* ids;
    int64_t ids_cap;
    int64_t* ids_count;
    int32_t skip_if_listed;     // tile kernels: exit when the list is complete
    int32_t cand_lds_acc;       // candidate kernel: S, A of all (shower, sphere) pairs in LDS
    int32_t shower_lds;         // listed kernels: the per-shower table in LDS
};

// Per shower, for the listed kernels: first step, counter-word base (the counter
// word of step i is ctr_base + i without caller step ids), t_ref and the shower id.
struct ShowerRec {
    int64_t first;
    int64_t ctr_base;
    double t_ref;
    uint32_t id;
    uint32_t pad;
};


__device__ __forceinline__ bool soft_list_complete(const SoftArgs& sa)
{
    const int64_t n = *sa.ids_count;
    return n >= 0 && n <= sa.ids_cap;
}

struct alignas(16) SoftStep {
    double x0, y0, h0, t0, u, v, w;
    double cos_t, sin_t, photons, ds, inv_bc;
    double b1x, b1y, b1z, b2x, b2y, b2z;
    double r2, g1, f_m, kl_nb;
    double g_cos, g_sin, g_phot;     // adjoint accumulators of the step
    int32_t i_m, boff, sidx;
    uint32_t ctr1;                   // counter word 1 of the step's random numbers
};
static_assert(sizeof(SoftStep) % 16 == 0, "soft step entry alignment");

constexpr int kSoftTS = 32;
// forward: 8 waves (<= 256 VGPRs, two waves per SIMD); adjoint: 4 waves, whose
// reverse sweep needs more registers than two waves per SIMD leave
// 8 waves for both: the adjoint at 4 waves keeps 288 registers (one wave per SIMD);
// built for 8 it gets 256 (two per SIMD) at the cost of a few spills, which is faster
__host__ __device__ constexpr int soft_max_waves(int mode) { return mode == 0 ? 8 : 8; }
// adjoint bins (dL/dpsi_i, dL/dP_j(h_i)) of the lowest kSoftBinNodes nodes live in
// LDS (h_obs + 51 km on a 50 m grid); the rare contributions above go to HBM
constexpr int kSoftBinNodes = 1024;

__host__ __device__ inline int soft_bin_nodes(int n_nodes)
{
    return n_nodes < kSoftBinNodes ? n_nodes : kSoftBinNodes;
}

// per wave: step stash, flag row and (forward only) S, A per telescope
__host__ __device__ inline size_t soft_wave_bytes(int mode, int n_tel)
{
    return kSoftTS * sizeof(SoftStep) + kWave * sizeof(int32_t) +
           (mode == 0 ? (size_t)2 * n_tel * sizeof(double) : 0);
}

// per workgroup: adjoint bins, then {X, Y, R^2, 1 / (2 R sigma)} per telescope, then the waves
// node records {psi, P1..P5} of the lowest kSoftNodeLds nodes staged in LDS for the
// bunch lookups of the forward and of the listed adjoint
constexpr int kSoftNodeLds = 1024;

__host__ __device__ inline int soft_node_lds(int n_nodes)
{
    return n_nodes < kSoftNodeLds ? n_nodes : kSoftNodeLds;
}

__host__ __device__ inline size_t soft_lds_bytes(int mode, int n_nodes, int n_tel, int waves)
{
    const size_t bins = mode == 1 ? (size_t)6 * soft_bin_nodes(n_nodes) * sizeof(double) : 0;
    const size_t nodes = mode == 0 ? (size_t)kNode64 * soft_node_lds(n_nodes) * sizeof(double) : 0;
    return bins + (size_t)n_tel * 4 * sizeof(double) + nodes + (size_t)waves * soft_wave_bytes(mode, n_tel);
}

// step setup with a frozen bunch count; false when the step emits nothing
__device__ inline bool soft_step_setup(const Args& a, int64_t i, int64_t nb, SoftStep& e,
                                       const double* node_lds = nullptr, int n_lds = 0)
{
    // no contraction: the threshold decision is the one of the FP64 definition and
    // of the screening pass's step setup
#pragma clang fp contract(off)
    const double x0 = a.x0[i], y0 = a.y0[i], h0 = a.h0[i];
    const double u = a.u[i], v = a.v[i], w = a.w[i];
    const double L = a.len[i], t0 = a.t0[i], E = a.energy[i];
    const double m = a.ptype[i] == CKV_MUON ? kMassMuon : kMassElectron;
    // every test evaluated (no short circuit) and the mass inside one of them (E c
    // with c = m / 1 GeV in (0, 1) is finite exactly when E is): all the step's loads
    // go out in one round
    const int n_finite = (int)isfinite(x0) + (int)isfinite(y0) + (int)isfinite(h0) + (int)isfinite(u) +
                         (int)isfinite(v) + (int)isfinite(w) + (int)isfinite(L) + (int)isfinite(t0) +
                         (int)isfinite(E * (m * 1e-3));
    if (n_finite != 9 || !(L > 0.0) || nb <= 0) return false;
    const double r = m / E;
    const double r2 = r * r;
    if (!(r2 < 1.0)) return false;
    const double h_mid = h0 - (0.5 * L) * w;
    const double hc = h_mid < a.h_obs ? a.h_obs : (h_mid > a.h_top ? a.h_top : h_mid);
    const double x = (hc - a.h_obs) * a.inv_step;
    int64_t im = (int64_t)floor(x);
    if (im > a.n_nodes - 2) im = a.n_nodes - 2;
    const double fm = x - (double)im;
    // psi at the two nodes: from the LDS copy of the lowest nodes when it holds them
    double lo, hi;
    if (im + 1 < n_lds) {
        lo = as_lds(node_lds)[kNode64 * im];
        hi = as_lds(node_lds)[kNode64 * (im + 1)];
    } else {
        lo = as_hbm(a.node64)[kNode64 * im];
        hi = as_hbm(a.node64)[kNode64 * (im + 1)];
    }
    const double psi = lo + fm * (hi - lo);
    const double n2 = 1.0 + psi;
    const double num = psi - n2 * r2;
    if (!(num > 0.0)) return false;
    // past the threshold test the step's values take reciprocals from the hardware
    // estimate and two Newton steps (within an ulp or two of the quotient): nothing
    // decides on them, and S, A and the gradient move by a few ulps at most
    e.g1 = (1.0 - r2) * n2;
    const double sin2 = num * rcp64(e.g1);
    const double nbd = (double)nb;
    const double inv_nb = rcp64(nbd);
    e.x0 = x0; e.y0 = y0; e.h0 = h0; e.t0 = t0; e.u = u; e.v = v; e.w = w;
    e.kl_nb = (a.k_ft * L) * inv_nb;
    e.photons = e.kl_nb * sin2;
    e.cos_t = rcp64(sqrt(e.g1));
    e.sin_t = sqrt(sin2);
    e.ds = L * inv_nb;
    e.inv_bc = rcp64(sqrt(1.0 - r2) * kSpeedOfLight);
    const double Dx = u, Dy = v, Dz = -w;
    const double sgn = copysign(1.0, Dz);
    const double ia = -rcp64(sgn + Dz);
    const double ib = Dx * Dy * ia;
    e.b1x = 1.0 + sgn * Dx * Dx * ia;
    e.b1y = sgn * ib;
    e.b1z = -sgn * Dx;
    e.b2x = ib;
    e.b2y = sgn + Dy * Dy * ia;
    e.b2z = -Dy;
    e.r2 = r2;
    e.f_m = fm;
    e.i_m = (int32_t)im;
    e.g_cos = e.g_sin = e.g_phot = 0.0;
    return true;
}

// One bunch k of a soft-response step e (its random numbers from the counter
// (k, seg_id, shower_id, 0)): emission, propagation and the soft weights over
// the candidate spheres.  MODE 0 adds photons * Phi and photons * Phi * t into
// acc (LDS, S then A per telescope); MODE 1 runs the adjoint of the bunch into
// the table bins and g_psi0 and returns the step-level adjoints (dL/dcos_t,
// dL/dsin_t, dL/dphotons) in o_cos, o_sin, o_phot.  Returns true when some
// sphere has z >= -kSoftZCut, i.e. the bunch enters S, A and the gradient.
// NODE_LDS: node records of the lowest n_lds nodes come from node_lds (LDS).
template <int MODE, bool NODE_LDS, bool ACC_LDS, typename AddBin>
__device__ __forceinline__ bool soft_bunch(const Args& a, const SoftArgs& sa, const SoftStep& e,
                                           int32_t k, uint32_t seg_id, uint32_t shower_id, int s,
                                           double t_ref, const double* tsh, double* acc,
                                           double* accA, AddBin& add_bin, double inv_nobs,
                                           double half_inv_nobs3,
                                           const double* node_lds, int n_lds,
                                           double& g_psi0, double& o_cos, double& o_sin,
                                           double& o_phot)
{
    const int N = a.n_nodes;
    constexpr double a1 = -0.5, a2 = 0.375, a3 = -0.3125, a4 = 0.2734375;
    const double ak[5] = {1.0, a1, a2, a3, a4};
    const double inv_c = 1.0 / kSpeedOfLight;
    constexpr double inv_sqrt2 = 0.70710678118654752440;
    constexpr double inv_sqrt2pi = 0.39894228040143267794;
    uint32_t r[4];
    philox4x32_10((uint32_t)k, seg_id, shower_id, 0u, a.key0, a.key1, r);
    const double u0 = ((double)r[0] + 0.5) * 2.3283064365386963e-10;
    const double s_along = ((double)k + u0) * e.ds;
    const double xe = e.x0 + s_along * e.u;
    const double ye = e.y0 + s_along * e.v;
    const double he = e.h0 - s_along * e.w;
    const double te = e.t0 + s_along * e.inv_bc;
    double sp, cp;
    sincos_turns64(r[1], sp, cp);
    const double Ex = cp * e.b1x + sp * e.b2x;
    const double Ey = cp * e.b1y + sp * e.b2y;
    const double Ez = cp * e.b1z + sp * e.b2z;
    const double pu = e.cos_t * e.u + e.sin_t * Ex;
    const double pv = e.cos_t * e.v + e.sin_t * Ey;
    const double pw = e.cos_t * e.w - e.sin_t * Ez;
    if (he < a.h_obs || he >= a.h_top || pw <= a.w_min) return false;
    // atmosphere at emission
    const double x = (he - a.h_obs) * a.inv_step;
    int ie = (int)x;
    ie = min(ie, N - 2);
    const double fe = x - (double)ie;
    double pa, pb, X1, X2, X3, X4, X5;
    if (NODE_LDS) {
        // the cell from the LDS copy when it holds it, else from HBM, each through
        // its own address space (no generic load)
        if (ie + 1 < n_lds) {
            const LdsF64* nl = as_lds(node_lds) + (size_t)kNode64 * ie;
            pa = nl[0]; X1 = nl[1]; X2 = nl[2]; X3 = nl[3]; X4 = nl[4]; X5 = nl[5];
            pb = nl[kNode64];
        } else {
            const HbmF64* nd = as_hbm(a.node64) + (size_t)kNode64 * ie;
            pa = nd[0]; X1 = nd[1]; X2 = nd[2]; X3 = nd[3]; X4 = nd[4]; X5 = nd[5];
            pb = nd[kNode64];
        }
    } else {
        const double* nd = a.node64 + (size_t)kNode64 * ie;
        pa = nd[0]; X1 = nd[1]; X2 = nd[2]; X3 = nd[3]; X4 = nd[4]; X5 = nd[5];
        pb = nd[kNode64];
    }
    const double psi_e = pa + fe * (pb - pa);
    const double dz = fe * a.step;
    const double dh = he - a.h_obs;
    // D_k = int (psi - psi_e)^k dh: node moments shifted to psi_e (Pascal
    // triangle, P_0(h_i) = h_i - h_obs) plus the in-cell part of the linear
    // profile, dz (psi_i - psi_e)^k / (k+1)
    const double c = -psi_e, del = pa - psi_e;
    const double X0 = (double)ie * a.step;
    X5 += c * X4; X4 += c * X3; X3 += c * X2; X2 += c * X1; X1 += c * X0;
    X5 += c * X4; X4 += c * X3; X3 += c * X2; X2 += c * X1;
    X5 += c * X4; X4 += c * X3; X3 += c * X2;
    X5 += c * X4; X4 += c * X3;
    X5 += c * X4;
    const double dl2 = del * del, dl3 = dl2 * del, dl4 = dl3 * del;
    double D[6];
    D[0] = dh;
    D[1] = X1 + dz * 0.5 * del;
    D[2] = X2 + dz * (1.0 / 3.0) * dl2;
    D[3] = X3 + dz * 0.25 * dl3;
    D[4] = X4 + dz * 0.2 * dl4;
    D[5] = X5 + dz * (1.0 / 6.0) * (dl4 * del);
    const double ne2 = 1.0 + psi_e;
    const double ne = sqrt(ne2);
    const double inv_ne = rcp64(ne), inv_pw = rcp64(pw);
    const double q = (inv_pw * inv_pw) * (inv_ne * inv_ne);
    const double Sser = D[0] + q * (a1 * D[1] + q * (a2 * D[2] + q * (a3 * D[3] + q * a4 * D[4])));
    const double U = (ne2 * D[0] + D[1]) +
                     q * (a1 * (ne2 * D[1] + D[2]) +
                          q * (a2 * (ne2 * D[2] + D[3]) +
                               q * (a3 * (ne2 * D[3] + D[4]) + q * a4 * (ne2 * D[4] + D[5]))));
    const double T = U * inv_ne * inv_pw * inv_c;
    const double adv = Sser * inv_pw;
    const double xg = xe + pu * adv;
    const double yg = ye + pv * adv;
    const double tt = te + T - t_ref;
    const double uo = pu * ne * inv_nobs;
    const double vo = pv * ne * inv_nobs;
    const double p = e.photons;

    // soft weights over candidate spheres
    double g_xg = 0, g_yg = 0, g_uo = 0, g_vo = 0, g_t = 0, g_p = 0;
    bool seen = false;
    int cur = 0, cend = 0;
    int first = -1;          // the cell's first sphere, known without a list read
    bool brute = false;
    const double wo2 = 1.0 - uo * uo - vo * vo;
    if (wo2 >= kLevelW2[0]) {
        const double fx = (xg - sa.gx0) * sa.inv_cell, fy = (yg - sa.gy0) * sa.inv_cell;
        if (fx >= 0.0 && fy >= 0.0 && fx < (double)sa.nx && fy < (double)sa.ny) {
            const int cidx = grid_level(wo2) * sa.level_cells + (int)fx * sa.ny + (int)fy;
            const uint2 ce = sa.cell_ent[cidx];
            cur = (int)ce.x;
            cend = cur + (int)(ce.y & 0xFFFFu);
            first = (int)(ce.y >> 16);
        }
    } else {
        brute = true;
        cend = a.n_tel;
    }
    for (; cur < cend; ++cur) {
        const int kt = brute ? cur : (first >= 0 ? first : (int)sa.cell_list[cur]);
        first = -1;
        const double* tp = tsh + 4 * kt;                  // LDS
        const double dx = xg - tp[0], dy = yg - tp[1];
        const double b = dx * uo + dy * vo;
        const double rho2 = dx * dx + dy * dy - b * b;
        const double z = (tp[2] - rho2) * tp[3];
        if (z < -kSoftZCut) continue;
        seen = true;
        const double W = 0.5 * erfc(-z * inv_sqrt2);
        if (MODE == 0) {
            if (ACC_LDS) {
                lds_add(&acc[kt], p * W);
                lds_add(&accA[kt], p * W * tt);
            } else {
                hbm_add(&acc[kt], p * W);
                hbm_add(&accA[kt], p * W * tt);
            }
        } else {
            const double gSk = sa.gS[(int64_t)s * a.n_tel + kt];
            const double gAk = sa.gA[(int64_t)s * a.n_tel + kt];
            g_p += gSk * W + gAk * W * tt;
            g_t += gAk * p * W;
            const double g_z = (gSk * p + gAk * p * tt) * inv_sqrt2pi * exp(-0.5 * z * z);
            const double g_r2 = -g_z * tp[3];
            g_xg += g_r2 * (2.0 * dx - 2.0 * b * uo);
            g_yg += g_r2 * (2.0 * dy - 2.0 * b * vo);
            g_uo += g_r2 * (-2.0 * b * dx);
            g_vo += g_r2 * (-2.0 * b * dy);
        }
    }
    if (MODE == 1 && (g_xg != 0.0 || g_yg != 0.0 || g_uo != 0.0 || g_vo != 0.0 || g_t != 0.0 ||
                      g_p != 0.0)) {
        // ---- reverse through propagation
        double g_pu = g_uo * ne * inv_nobs + g_xg * adv;
        double g_pv = g_vo * ne * inv_nobs + g_yg * adv;
        double g_ne = (g_uo * pu + g_vo * pv) * inv_nobs;
        // n_obs = sqrt(1 + psi_0): d(1/n_obs)/d psi_0 = -1 / (2 n_obs^3)
        g_psi0 -= (g_uo * pu + g_vo * pv) * ne * half_inv_nobs3;
        const double g_U = g_t * inv_c * inv_ne * inv_pw;
        g_ne -= g_t * T * inv_ne;
        double g_pw = -g_t * T * inv_pw;
        const double XS = g_xg * pu + g_yg * pv;
        const double g_S = XS * inv_pw;
        g_pw -= XS * adv * inv_pw;
        const double qk[5] = {1.0, q, q * q, q * q * q, q * q * q * q};
        double gD[6] = {0, 0, 0, 0, 0, 0};
        double g_q = 0.0;
        for (int kk = 0; kk < 5; ++kk) {
            const double akq = ak[kk] * qk[kk];
            gD[kk] += g_S * akq + g_U * akq * ne2;
            gD[kk + 1] += g_U * akq;
            if (kk >= 1)
                g_q += (g_S * D[kk] + g_U * (ne2 * D[kk] + D[kk + 1])) * (double)kk * ak[kk] * qk[kk - 1];
        }
        double g_ne2 = g_U * Sser;
        g_ne2 -= g_q * q * inv_ne * inv_ne;
        g_pw -= 2.0 * g_q * q * inv_pw;
        g_ne2 += g_ne * 0.5 * inv_ne;
        // D_k as a function of (P_j(h_i), psi_i, psi_e):
        //   dD_k/dpsi_e = -k D_{k-1} + dz del^(k-1) / (k+1)
        //   dD_k/dpsi_i = dz k del^(k-1) / (k+1)
        const double dpow[5] = {1.0, del, dl2, dl3, dl4};
        double g_psie = g_ne2, g_pa = 0.0;
#pragma unroll
        for (int kk = 1; kk <= 5; ++kk) {
            const double inc = dz * dpow[kk - 1] * (1.0 / (double)(kk + 1));
            g_psie += gD[kk] * (inc - (double)kk * D[kk - 1]);
            g_pa += gD[kk] * ((double)kk * inc);
        }
        // dL/dP_j(h_i): the Pascal shift transposed
        double G1 = gD[1], G2 = gD[2], G3 = gD[3], G4 = gD[4], G5 = gD[5];
        G4 += c * G5;
        G3 += c * G4; G4 += c * G5;
        G2 += c * G3; G3 += c * G4; G4 += c * G5;
        G1 += c * G2; G2 += c * G3; G3 += c * G4; G4 += c * G5;
        G1 += c * G2; G2 += c * G3; G3 += c * G4; G4 += c * G5;
        add_bin(1, ie, G1);
        add_bin(2, ie, G2);
        add_bin(3, ie, G3);
        add_bin(4, ie, G4);
        add_bin(5, ie, G5);
        add_bin(0, ie, g_pa + (1.0 - fe) * g_psie);
        add_bin(0, ie + 1, fe * g_psie);
        // ---- reverse through the direction on the cone and the yield
        const double g_cos = g_pu * e.u + g_pv * e.v + g_pw * e.w;
        const double g_sin = g_pu * Ex + g_pv * Ey - g_pw * Ez;
        o_cos = g_cos;
        o_sin = g_sin;
        o_phot = g_p;
    }
    return seen;
}

// Step-level part of the soft adjoint: dL/dcos_t, dL/dsin_t and dL/dphotons of
// bunches of step es to dL/dpsi at the two table nodes around the step's
// midpoint (cos_t = g1^(-1/2), sin^2 = 1 - 1/g1, g1 = (1 - r^2) n^2; linear in
// the three inputs, so per-bunch and per-step application agree).
template <typename AddBin>
__device__ __forceinline__ void soft_step_reverse(const SoftStep& es, double g_cos, double g_sin,
                                                  double g_phot, AddBin& add_bin)
{
    const double sin2 = es.sin_t * es.sin_t;
    double g_sin2 = g_phot * es.kl_nb;
    if (sin2 > 0.0) g_sin2 += g_sin / (2.0 * es.sin_t);
    const double g_g1 = -0.5 * g_cos * es.cos_t * es.cos_t * es.cos_t + g_sin2 / (es.g1 * es.g1);
    const double g_psim = g_g1 * (1.0 - es.r2);
    if (g_psim != 0.0) {
        add_bin(0, es.i_m, (1.0 - es.f_m) * g_psim);
        add_bin(0, es.i_m + 1, es.f_m * g_psim);
    }
}

template <int MODE>
__global__ void __launch_bounds__(soft_max_waves(MODE) * kWave) soft_kernel(Args a, SoftArgs sa)
{
    extern __shared__ __align__(16) unsigned char lds[];
    // with a complete list soft_list_kernel (adjoint) or soft_cand_kernel (forward
    // after the screening pass) does the work (the same decision in every thread)
    if (sa.skip_if_listed && soft_list_complete(sa)) return;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int N = a.n_nodes;
    const int NB = soft_bin_nodes(N);
    double* bins = reinterpret_cast<double*>(lds);                 // MODE 1: 6 x NB
    double* tsh = bins + (MODE == 1 ? 6 * NB : 0);     // n_tel x {X, Y, R^2, 1 / (2 R sigma)}
    double* nlds = tsh + 4 * a.n_tel;                 // MODE 0: lowest node records
    const int NL = soft_node_lds(N);
    unsigned char* wbase = reinterpret_cast<unsigned char*>(nlds + (MODE == 0 ? kNode64 * NL : 0)) +
                           (size_t)wave * soft_wave_bytes(MODE, a.n_tel);
    SoftStep* stash = reinterpret_cast<SoftStep*>(wbase);
    int32_t* flags = reinterpret_cast<int32_t*>(wbase + kSoftTS * sizeof(SoftStep));
    double* acc = reinterpret_cast<double*>(flags + kWave);     // MODE 0: S then A per telescope
    if (MODE == 1)
        for (int q = threadIdx.x; q < 6 * NB; q += blockDim.x) bins[q] = 0.0;
    for (int q = threadIdx.x; q < a.n_tel; q += blockDim.x) {
        tsh[4 * q] = a.tel[4 * q];
        tsh[4 * q + 1] = a.tel[4 * q + 1];
        tsh[4 * q + 2] = a.tel[4 * q + 3];
        tsh[4 * q + 3] = 1.0 / (2.0 * a.tel[4 * q + 2] * sa.sigma);
    }
    if (MODE == 0)
        for (int q = threadIdx.x; q < kNode64 * NL; q += blockDim.x) nlds[q] = a.node64[q];
    if (MODE == 0)
        for (int q = lane; q < 2 * a.n_tel; q += kWave) acc[q] = 0.0;
    flags[lane] = 0;
    __syncthreads();
    // j = 0: dL/dpsi_i, j = 1..5: dL/dP_j(h_i)
    auto add_bin = [&](int j, int i, double v) {
        if (i < NB) lds_add(&bins[j * NB + i], v);
        else hbm_add(j == 0 ? &sa.g_psi[i] : &sa.g_P[(size_t)(j - 1) * N + i], v);
    };

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t le_mask = lt_mask | (1ull << lane);
    const double inv_nobs = 1.0 / a.n_obs;
    const double half_inv_nobs3 = 0.5 * inv_nobs * inv_nobs * inv_nobs;
    double g_psi0 = 0.0;
    const int64_t n_tiles = a.ctrl[kNumTiles];

    for (;;) {
        int64_t t = 0;
        if (lane == 0) t = (int64_t)atomicAdd((unsigned long long*)&a.ctrl[kTileCounter], 1ull);
        t = uniform(t);
        if (t >= n_tiles) break;
        int lo = 0, hi = a.n_showers;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.tiles_before[mid] <= t) lo = mid; else hi = mid;
        }
        const int s = lo;
        const int64_t sfirst = a.seg_offsets[s];
        const int64_t g0 = a.shower_first[s] + (t - a.tiles_before[s]) * (int64_t)kSoftTS;
        const int64_t gend = min(g0 + (int64_t)kSoftTS, a.seg_offsets[s + 1]);
        const int nseg = (int)(gend - g0);
        const uint32_t shower_id = a.shower_ids ? a.shower_ids[s] : (uint32_t)s;
        const int64_t seg_id0 = (a.seg_id_base ? a.seg_id_base[s] : 0) + (g0 - sfirst);
        const double t_ref = a.t_ref[s];

        SoftStep st;
        int64_t nb = 0;
        bool emits = false;
        double len = 0.0;
        if (lane < nseg) {
            const int64_t nbf = sa.nb_frozen[g0 + lane];
            len = a.len[g0 + lane];
            emits = soft_step_setup(a, g0 + lane, nbf, st);
            if (emits) nb = nbf;
        }
        // the tile limit on the frozen counts, then the cull of the steps whose
        // bunches can weight no sphere (screen_annulus, as in the screening pass)
        if (wave_last(wave_incl_scan(nb)) >= ((int64_t)1 << 30)) {
            if (lane == 0 && a.result) atomicOr(&a.result->error, 2);
            continue;
        }
        if (a.cull_rmax > 0.0) {
            double cgx = 0.0, cgy = 0.0, cmid = 0.0, chalf = -1.0;
            const int ok = emits && screen_annulus(a, st.x0, st.y0, st.h0, st.u, st.v, st.w, len, st.cos_t,
                                                   st.sin_t, cgx, cgy, cmid, chalf) ? 1 : 0;
            // (called by the whole wave: the upper half-wave tests spheres for the lower one)
            const bool reached = annulus_holds_centre<4>(tsh, a.n_tel, lane, ok, cgx, cgy, cmid, chalf);
            if (ok && !reached) {
                emits = false;
                nb = 0;
            }
        }
        const int64_t incl = wave_incl_scan(nb);
        const int64_t total = wave_last(incl);
        const uint64_t emit_mask = __ballot(emits);
        const int excl = (int)(incl - nb);
        if (emits) {
            st.boff = excl;
            st.sidx = lane;
            st.ctr1 = a.step_id ? a.step_id[g0 + lane] : (uint32_t)(seg_id0 + lane);
            stash[__popcll(emit_mask & lt_mask)] = st;
        }
        wave_lds_sync();

        for (int64_t c0 = 0; c0 < total; c0 += kWave) {
            const int32_t j = (int32_t)(c0 + lane);
            const bool active = j < total;
            const int cnt0 = __popcll(__ballot(emits && excl <= (int)c0));
            if (emits && excl > (int)c0 && excl < (int)c0 + kWave) flags[excl - (int)c0] = 1;
            wave_lds_sync();
            const uint64_t starts = __ballot(flags[lane] != 0);
            flags[lane] = 0;
            const int si = cnt0 - 1 + __popcll(starts & le_mask);
            if (active) {
                SoftStep& e = stash[si];
                const int32_t k = j - e.boff;
                double o_cos = 0.0, o_sin = 0.0, o_phot = 0.0;
                soft_bunch<MODE, MODE == 0, true>(a, sa, e, k, e.ctr1, shower_id,
                                                   s, t_ref, tsh, acc, acc + a.n_tel, add_bin, inv_nobs,
                                                   half_inv_nobs3, nlds, NL, g_psi0, o_cos, o_sin,
                                                   o_phot);
                if (MODE == 1 && (o_cos != 0.0 || o_sin != 0.0 || o_phot != 0.0)) {
                    lds_add(&e.g_cos, o_cos);
                    lds_add(&e.g_sin, o_sin);
                    lds_add(&e.g_phot, o_phot);
                }
            }
        }
        wave_lds_sync();
        if (MODE == 0) {
            for (int kk = lane; kk < a.n_tel; kk += kWave) {
                const double vs = acc[kk], va = acc[a.n_tel + kk];
                if (vs != 0.0) atomicAdd(&sa.S[(int64_t)s * a.n_tel + kk], vs);
                if (va != 0.0) atomicAdd(&sa.A[(int64_t)s * a.n_tel + kk], va);
                acc[kk] = 0.0;
                acc[a.n_tel + kk] = 0.0;
            }
        } else if (emits) {
            // ---- reverse through the step setup (index at the step midpoint)
            const SoftStep& es = stash[__popcll(emit_mask & lt_mask)];
            soft_step_reverse(es, es.g_cos, es.g_sin, es.g_phot, add_bin);
        }
        wave_lds_sync();
    }
    if (MODE == 1) {
        if (g_psi0 != 0.0) add_bin(0, 0, g_psi0);
        __syncthreads();
        for (int qq = threadIdx.x; qq < 6 * NB; qq += blockDim.x) {
            const double v = bins[qq];
            const int j = qq / NB, i = qq - j * NB;
            if (v != 0.0) atomicAdd(j == 0 ? &sa.g_psi[i] : &sa.g_P[(size_t)(j - 1) * N + i], v);
        }
    }
}

constexpr int kSoftListThreads = 512;   // listed adjoint: workgroup size
constexpr int kSoftCandThreads = 512;   // listed forward: workgroup size

// Listed bunches of a wave (consecutive list entries, one per lane; id is the
// lane's entry, loaded by the caller): the step setup and the shower lookup are
// done once per run of lanes that name the same step (the screening pass lists a
// step's bunches together) and passed to the run's other lanes by lane shuffles.
// shr: the per-shower table in LDS, or null (then from HBM); node_lds: the lowest
// n_lds node records in LDS.  REV: also the step-level values of the reverse sweep.
// True for lanes whose id names a bunch of the inputs on a step that gives light.
// Called by the whole wave.
template <bool REV>
__device__ __forceinline__ bool listed_setup(const Args& a, const SoftArgs& sa, uint64_t id, bool have,
                                             int lane, const ShowerRec* shr, const double* node_lds,
                                             int n_lds, SoftStep& e, int& shower, uint32_t& ctr1,
                                             uint32_t& shower_id, double& t_ref, int32_t& k)
{
    const int64_t i = have ? (int64_t)(id >> kSoftIdBits) : -1;
    k = (int32_t)(id & ((1u << kSoftIdBits) - 1));
    const bool named = have && i < a.n;
    const int64_t nbf = named ? sa.nb_frozen[i] : 0;
    const int64_t i_prev = __shfl_up(i, 1);
    const bool head = named && (lane == 0 || i_prev != i);
    int lit = 0, lo = 0;
    uint32_t c1 = 0, sid = 0;
    double tr = 0.0;
    if (head) {
        int hi = a.n_showers;                   // the shower holding step i
        if (shr) {
            // the LDS table through its own address space (no generic loads)
            using LdsRec = const __attribute__((address_space(3))) ShowerRec;
            LdsRec* sh = (LdsRec*)shr;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sh[mid].first <= i) lo = mid; else hi = mid;
            }
            c1 = a.step_id ? a.step_id[i] : (uint32_t)(sh[lo].ctr_base + i);
            sid = sh[lo].id;
            tr = sh[lo].t_ref;
        } else {
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.seg_offsets[mid] <= i) lo = mid; else hi = mid;
            }
            c1 = a.step_id ? a.step_id[i]
                           : (uint32_t)((a.seg_id_base ? a.seg_id_base[lo] : 0) + (i - a.seg_offsets[lo]));
            sid = a.shower_ids ? a.shower_ids[lo] : (uint32_t)lo;
            tr = a.t_ref[lo];
        }
        lit = soft_step_setup(a, i, nbf, e, node_lds, n_lds) ? 1 : 0;
    }
    // the run's head: the nearest head lane at or below this one
    const uint64_t heads = __ballot(head);
    const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
    const uint64_t mine = heads & le;
    const int src = mine ? 63 - __builtin_clzll(mine) : lane;
    lit = __shfl(lit, src);
    shower = __shfl(lo, src);
    ctr1 = __shfl(c1, src);
    shower_id = __shfl(sid, src);
    t_ref = __shfl(tr, src);
    e.x0 = __shfl(e.x0, src); e.y0 = __shfl(e.y0, src); e.h0 = __shfl(e.h0, src);
    e.t0 = __shfl(e.t0, src); e.u = __shfl(e.u, src); e.v = __shfl(e.v, src); e.w = __shfl(e.w, src);
    e.cos_t = __shfl(e.cos_t, src); e.sin_t = __shfl(e.sin_t, src);
    e.photons = __shfl(e.photons, src); e.ds = __shfl(e.ds, src); e.inv_bc = __shfl(e.inv_bc, src);
    e.b1x = __shfl(e.b1x, src); e.b1y = __shfl(e.b1y, src); e.b1z = __shfl(e.b1z, src);
    e.b2x = __shfl(e.b2x, src); e.b2y = __shfl(e.b2y, src); e.b2z = __shfl(e.b2z, src);
    if (REV) {
        e.r2 = __shfl(e.r2, src); e.g1 = __shfl(e.g1, src); e.f_m = __shfl(e.f_m, src);
        e.kl_nb = __shfl(e.kl_nb, src); e.i_m = __shfl(e.i_m, src);
    }
    return named && lit && k < nbf;
}

// Per-shower table of the listed kernels, staged into LDS by the workgroup.
__device__ __forceinline__ void stage_showers(const Args& a, ShowerRec* shr)
{
    for (int q = threadIdx.x; q < a.n_showers; q += blockDim.x) {
        ShowerRec r;
        r.first = a.seg_offsets[q];
        r.ctr_base = (a.seg_id_base ? a.seg_id_base[q] : 0) - a.seg_offsets[q];
        r.t_ref = a.t_ref[q];
        r.id = a.shower_ids ? a.shower_ids[q] : (uint32_t)q;
        r.pad = 0;
        shr[q] = r;
    }
}

// Adjoint over the forward's list: one listed bunch per thread, its step set up
// again (bunch count frozen), the bunch recomputed from its random numbers and
// reversed into the table bins, the step-level part applied per bunch.  Runs only
// when the list is complete; ids that do not name a bunch of the inputs are skipped.
__global__ void __launch_bounds__(kSoftListThreads) soft_list_kernel(Args a, SoftArgs sa)
{
    extern __shared__ __align__(16) unsigned char lds[];
    if (!soft_list_complete(sa)) return;
    const int64_t n_ids = *sa.ids_count;
    const int N = a.n_nodes;
    const int NB = soft_bin_nodes(N);
    double* bins = reinterpret_cast<double*>(lds);               // 6 x NB
    double* tsh = bins + 6 * NB;                                 // n_tel x {X, Y, R^2, 1 / (2 R sigma)}
    double* nlds = tsh + 4 * a.n_tel;                            // lowest node records
    const int NL = soft_node_lds(N);
    for (int q = threadIdx.x; q < 6 * NB; q += blockDim.x) bins[q] = 0.0;
    for (int q = threadIdx.x; q < kNode64 * NL; q += blockDim.x) nlds[q] = a.node64[q];
    for (int q = threadIdx.x; q < a.n_tel; q += blockDim.x) {
        tsh[4 * q] = a.tel[4 * q];
        tsh[4 * q + 1] = a.tel[4 * q + 1];
        tsh[4 * q + 2] = a.tel[4 * q + 3];
        tsh[4 * q + 3] = 1.0 / (2.0 * a.tel[4 * q + 2] * sa.sigma);
    }
    ShowerRec* shr = sa.shower_lds ? reinterpret_cast<ShowerRec*>(nlds + kNode64 * NL) : nullptr;
    if (shr) stage_showers(a, shr);
    __syncthreads();
    auto add_bin = [&](int j, int i, double v) {
        if (i < NB) lds_add(&bins[j * NB + i], v);
        else hbm_add(j == 0 ? &sa.g_psi[i] : &sa.g_P[(size_t)(j - 1) * N + i], v);
    };
    const double inv_nobs = 1.0 / a.n_obs;
    const double half_inv_nobs3 = 0.5 * inv_nobs * inv_nobs * inv_nobs;
    double g_psi0 = 0.0;
    const int lane = lane_id();
    // each lane's next list entry is loaded one round ahead, while the current
    // bunch is computed
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t q0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1));
    uint64_t id = q0 + lane < n_ids ? sa.ids[q0 + lane] : ~0ull;
    for (; q0 < n_ids; q0 += stride) {
        const int64_t q = q0 + lane;
        const uint64_t id_next = q + stride < n_ids ? sa.ids[q + stride] : ~0ull;
        SoftStep e;
        int lo;
        uint32_t seg_id, shower_id;
        double t_ref;
        int32_t k;
        if (listed_setup<true>(a, sa, id, q < n_ids, lane, shr, nlds, NL, e, lo, seg_id, shower_id,
                               t_ref, k)) {
            double o_cos = 0.0, o_sin = 0.0, o_phot = 0.0;
            soft_bunch<1, true, true>(a, sa, e, k, seg_id, shower_id, lo, t_ref, tsh, nullptr, nullptr,
                                add_bin, inv_nobs, half_inv_nobs3, nlds, NL, g_psi0, o_cos, o_sin,
                                o_phot);
            if (o_cos != 0.0 || o_sin != 0.0 || o_phot != 0.0)
                soft_step_reverse(e, o_cos, o_sin, o_phot, add_bin);
        }
        id = id_next;
    }
    if (g_psi0 != 0.0) add_bin(0, 0, g_psi0);
    __syncthreads();
    for (int qq = threadIdx.x; qq < 6 * NB; qq += blockDim.x) {
        const double v = bins[qq];
        const int j = qq / NB, i = qq - j * NB;
        if (v != 0.0) atomicAdd(j == 0 ? &sa.g_psi[i] : &sa.g_P[(size_t)(j - 1) * N + i], v);
    }
}

// Soft forward over the screening pass's candidate list: one candidate bunch per
// thread, its step set up again with the frozen count and the bunch recomputed in
// FP64 exactly as in the tile kernel; S and A are added straight into HBM.  Runs
// only when the list is complete; ids that name no bunch are skipped.
__global__ void __launch_bounds__(kSoftCandThreads) soft_cand_kernel(Args a, SoftArgs sa)
{
    extern __shared__ __align__(16) unsigned char lds[];
    if (!soft_list_complete(sa)) return;
    const int64_t n_ids = *sa.ids_count;
    const int N = a.n_nodes;
    double* tsh = reinterpret_cast<double*>(lds);                // n_tel x {X, Y, R^2, 1 / (2 R sigma)}
    double* nlds = tsh + 4 * a.n_tel;                            // lowest node records
    const int NL = soft_node_lds(N);
    for (int q = threadIdx.x; q < a.n_tel; q += blockDim.x) {
        tsh[4 * q] = a.tel[4 * q];
        tsh[4 * q + 1] = a.tel[4 * q + 1];
        tsh[4 * q + 2] = a.tel[4 * q + 3];
        tsh[4 * q + 3] = 1.0 / (2.0 * a.tel[4 * q + 2] * sa.sigma);
    }
    for (int q = threadIdx.x; q < kNode64 * NL; q += blockDim.x) nlds[q] = a.node64[q];
    // S and A summed per workgroup in LDS when they fit (added to HBM once at the
    // end): bunches near one sphere would otherwise all update the same two words
    const int64_t nsk = (int64_t)a.n_showers * a.n_tel;
    double* accS = nlds + kNode64 * NL;
    double* accA = accS + nsk;
    if (sa.cand_lds_acc)
        for (int64_t q = threadIdx.x; q < 2 * nsk; q += blockDim.x) accS[q] = 0.0;
    ShowerRec* shr = sa.shower_lds
                         ? reinterpret_cast<ShowerRec*>(sa.cand_lds_acc ? accA + nsk : accS)
                         : nullptr;
    if (shr) stage_showers(a, shr);
    __syncthreads();
    auto no_bins = [](int, int, double) {};
    const double inv_nobs = 1.0 / a.n_obs;
    const double half_inv_nobs3 = 0.5 * inv_nobs * inv_nobs * inv_nobs;
    double g_psi0 = 0.0;
    const int lane = lane_id();
    // each lane's next list entry is loaded one round ahead, while the current
    // bunch is computed
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t q0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1));
    uint64_t id = q0 + lane < n_ids ? sa.ids[q0 + lane] : ~0ull;
    for (; q0 < n_ids; q0 += stride) {
        const int64_t q = q0 + lane;
        const uint64_t id_next = q + stride < n_ids ? sa.ids[q + stride] : ~0ull;
        SoftStep e;
        int lo;
        uint32_t seg_id, shower_id;
        double t_ref;
        int32_t k;
        if (listed_setup<false>(a, sa, id, q < n_ids, lane, shr, nlds, NL, e, lo, seg_id, shower_id,
                                t_ref, k)) {
            double o_cos = 0.0, o_sin = 0.0, o_phot = 0.0;
            // S and A into the workgroup's LDS rows, or straight into HBM (a uniform
            // choice; each branch keeps its address space)
            if (sa.cand_lds_acc)
                soft_bunch<0, true, true>(a, sa, e, k, seg_id, shower_id, lo, t_ref, tsh,
                                          accS + (int64_t)lo * a.n_tel, accA + (int64_t)lo * a.n_tel, no_bins,
                                          inv_nobs, half_inv_nobs3, nlds, NL, g_psi0, o_cos, o_sin, o_phot);
            else
                soft_bunch<0, true, false>(a, sa, e, k, seg_id, shower_id, lo, t_ref, tsh,
                                           sa.S + (int64_t)lo * a.n_tel, sa.A + (int64_t)lo * a.n_tel, no_bins,
                                           inv_nobs, half_inv_nobs3, nlds, NL, g_psi0, o_cos, o_sin, o_phot);
        }
        id = id_next;
    }
    if (sa.cand_lds_acc) {
        __syncthreads();
        for (int64_t q = threadIdx.x; q < nsk; q += blockDim.x) {
            if (accS[q] != 0.0) atomicAdd(&sa.S[q], accS[q]);
            if (accA[q] != 0.0) atomicAdd(&sa.A[q], accA[q]);
        }
    }
}

__global__ void zero_kernel(double* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
namespace {

// Raises a kernel's dynamic-LDS limit the first time it is launched on a device
// (once per kernel and device; safe when several host threads launch).
void allow_lds(const void* kernel, int bytes)
{
    static std::mutex mu;
    static std::set<std::pair<const void*, int>> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert({kernel, dev}).second)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

Args make_args(const RunPlan& p)
{
    Args a{};
    const ckv_segments& s = p.segs;
    a.x0 = s.x0; a.y0 = s.y0; a.h0 = s.h0; a.u = s.u; a.v = s.v; a.w = s.w;
    a.len = s.length; a.t0 = s.t0; a.energy = s.energy; a.ptype = s.ptype; a.n = s.n;
    a.step_id = s.step_id;
    a.seg_offsets = p.showers.seg_offsets;
    a.t_ref = p.showers.t_ref;
    a.shower_ids = p.showers.shower_ids;
    a.seg_id_base = p.showers.seg_id_base;
    a.n_showers = p.showers.n_showers;
    const ckv_atmo* at = p.atmo;
    a.n_nodes = (int32_t)at->n_nodes;
    a.h_obs = at->h_obs; a.step = at->step; a.inv_step = at->inv_step; a.h_top = at->h_top;
    a.n_obs = at->n_obs;
    a.node64 = at->d_node64;
    a.cell32 = at->d_cell32;
    a.lds_entries = lds_entries(p.params.precision, a.n_nodes, p.prof_bins > 0);
    a.hnodes = at->d_hnodes;
    a.search_pow2 = 0;
    while ((a.search_pow2 ? 2 * a.search_pow2 : 1) < a.n_nodes - 1)
        a.search_pow2 = a.search_pow2 ? 2 * a.search_pow2 : 1;
    a.depth = at->d_depth;
    if (p.prof_bins > 0) {
        a.prof_ph = p.out.profile_photons;
        a.prof_bu = p.out.profile_bunches;
        a.inv_bin = 1.0 / p.params.depth_bin_gcm2;
        a.prof_bins = p.prof_bins;
    }
    const ckv_array* ar = p.arr;
    if (ar) {
        a.n_tel = ar->n_tel;
        a.tel = ar->d_tel;
        a.gx0 = ar->hit.gx0; a.gy0 = ar->hit.gy0; a.inv_cell = ar->hit.inv_cell;
        a.nx = ar->hit.nx; a.ny = ar->hit.ny; a.level_cells = ar->hit.level_cells;
        a.cell_off = ar->hit.d_cell_off;
        a.cell_list = ar->hit.d_cell_list;
        a.cell_ent = reinterpret_cast<const uint2*>(ar->hit.d_cell_ent);
    }
    a.bunch_size = p.params.bunch_size;
    a.k_ft = p.k_ft;
    a.inv_l1 = 1.0 / p.params.lambda_min_nm;
    a.dl = 1.0 / p.params.lambda_min_nm - 1.0 / p.params.lambda_max_nm;
    a.w_min = p.params.w_min;
    a.grazing_exact = p.params.grazing_exact;
    a.earth_r = p.params.earth_radius_m;
    a.r_obs = a.earth_r + a.h_obs;
    a.key0 = (uint32_t)p.params.seed;
    a.key1 = (uint32_t)(p.params.seed >> 32);
    a.tile_segs = p.tile_segs;
    a.cur_step = p.cursor.step;
    a.cur_shower = p.cursor.shower;
    a.ctrl = p.ctrl;
    a.tiles_before = p.tiles_before;
    a.blocks_before = p.blocks_before;
    a.shower_first = p.shower_first;
    a.tile_run_off = p.tile_run_off;
    a.tile_run_n = p.tile_run_n;
    a.tile_hits = p.tile_hits;
    a.runs = p.runs;
    a.run_cap = p.run_cap;
    a.block_hits = p.block_hits;
    a.block_sums = p.block_sums;
    a.shower_tel = p.shower_tel;
    a.stage_fill = p.stage_fill;
    a.stage = p.stage;
    a.stage_blocks = p.stage_slots / kStageBlock;
    a.max_tiles = p.max_tiles;
    a.max_row_blocks = p.max_row_blocks;
    a.records = p.out.records;
    a.ids = p.out.ids;
    a.capacity = p.out.capacity;
    a.tel_offsets = p.out.tel_offsets;
    a.result = p.out.result;
    return a;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return CKV_ERR_HIP;
    }
    return CKV_OK;
}

}  // namespace

int emit_config(int precision, int n_tel, int prof_bins, const ckv_atmo* atmo, int tile_segs,
                int max_waves, int* waves, size_t* lds_bytes, bool narrow_ok)
{
    const size_t srch = atmo->h_nodes.empty() ? 0 : search_bytes((int)atmo->n_nodes);
    const size_t cap = 160 * 1024;
    const size_t per = wave_bytes(precision, tile_segs, n_tel, prof_bins);
    // FP64: 16 waves only as the narrow build (partial table), else at most 8
    if (precision == 0 && !narrow_ok) max_waves = std::min(max_waves, kMaxEmitWaves / 2);
    for (int wv = kMaxEmitWaves; wv >= 1; wv /= 2) {
        if (wv > max_waves) continue;
        const bool partial = prof_bins > 0 || (precision == 0 && wv > kMaxEmitWaves / 2);
        const size_t tab =
            ((table_bytes(precision, (int)atmo->n_nodes, partial) + 15) & ~(size_t)15) + srch;
        const size_t tot = tab + tel_bytes(n_tel) + (size_t)wv * per;
        if (tot <= cap) {
            *waves = wv;
            *lds_bytes = tot;
            return CKV_OK;
        }
    }
    set_error("atmosphere table too large for LDS");
    return CKV_ERR_TABLE;
}

namespace {

template <int PREC, int TS, int FEAT>
int launch_emit(const Args& a, int grid, int waves, size_t lds, hipStream_t st)
{
    allow_lds((const void*)emit_kernel<PREC, TS, FEAT>, 160 * 1024);
    emit_kernel<PREC, TS, FEAT><<<grid, waves * kWave, lds, st>>>(a);
    return check_launch("emit");
}

template <int PREC, int TS>
int launch_emit_feat(const Args& a, int grid, int waves, size_t lds, hipStream_t st)
{
    if (a.hnodes) {
        // node tables run alone (checked by the caller) and with 32-step tiles
        if (TS == 32) return launch_emit<PREC, 32, kFeatSearch>(a, grid, waves, lds, st);
        set_error("node tables need tile_segments 32");
        return CKV_ERR_ARG;
    }
    if (a.earth_r > 0.0) {
        // the curved atmosphere runs alone (checked by the caller) and with 32-step tiles
        if (TS == 32) return launch_emit<PREC, 32, kFeatCurved>(a, grid, waves, lds, st);
        set_error("the curved atmosphere needs tile_segments 32");
        return CKV_ERR_ARG;
    }
    const int feat = (a.prof_bins > 0 ? kFeatProfile : 0) | (a.grazing_exact ? kFeatExact : 0);
    if constexpr (PREC == 0) {
        if (waves > emit_threads(0, 0) / kWave) {
            if (feat == 0) return launch_emit<PREC, TS, kFeatNarrow>(a, grid, waves, lds, st);
            set_error("the FP64 kernel runs 16 waves per workgroup only without other features");
            return CKV_ERR_ARG;
        }
    }
    if constexpr (PREC == 1) {
        if (waves <= emit_threads(1, kFeatWide) / kWave) {
            if (feat == 0) return launch_emit<PREC, TS, kFeatWide>(a, grid, waves, lds, st);
            if (feat == kFeatProfile)
                return launch_emit<PREC, TS, kFeatProfile | kFeatWide>(a, grid, waves, lds, st);
        }
    }
    switch (feat) {
        case 0: return launch_emit<PREC, TS, 0>(a, grid, waves, lds, st);
        case kFeatProfile: return launch_emit<PREC, TS, kFeatProfile>(a, grid, waves, lds, st);
        case kFeatExact: return launch_emit<PREC, TS, kFeatExact>(a, grid, waves, lds, st);
        default: return launch_emit<PREC, TS, kFeatProfile | kFeatExact>(a, grid, waves, lds, st);
    }
}

template <int PREC>
int launch_emit_ts(const Args& a, int ts, int grid, int waves, size_t lds, hipStream_t st)
{
    switch (ts) {
        case 8: return launch_emit_feat<PREC, 8>(a, grid, waves, lds, st);
        case 16: return launch_emit_feat<PREC, 16>(a, grid, waves, lds, st);
        case 32: return launch_emit_feat<PREC, 32>(a, grid, waves, lds, st);
        case 64: return launch_emit_feat<PREC, 64>(a, grid, waves, lds, st);
    }
    set_error("tile_segments must be 8, 16, 32 or 64");
    return CKV_ERR_ARG;
}

}  // namespace

int launch_run(RunPlan& p)
{
    Args a = make_args(p);
    hipStream_t st = p.stream;
    init_kernel<<<1, 1024, 0, st>>>(a);
    if (int rc = check_launch("init")) return rc;
    int waves = 0;
    size_t lds = 0;
    int cap = p.emit_waves;
    if (p.params.precision == 1 && (p.params.grazing_exact || p.params.earth_radius_m > 0.0))
        cap = std::min(cap, emit_threads(1, kFeatExact) / kWave);
    // the narrow FP64 build: plain runs (no profile, exact or curved path, node tables)
    const bool narrow_ok = p.params.precision == 0 && p.prof_bins == 0 && !p.params.grazing_exact &&
                           p.params.earth_radius_m <= 0.0 && p.atmo->h_nodes.empty();
    if (int rc = emit_config(p.params.precision, a.n_tel, p.prof_bins, p.atmo, p.tile_segs, cap, &waves,
                             &lds, narrow_ok))
        return rc;
    if (p.params.precision == 0 && waves > kMaxEmitWaves / 2)
        a.lds_entries = lds_entries(0, a.n_nodes, true);
    if (p.prof_bins > 0) {
        // the profile accumulates by atomics: clear it (a kernel, so the run stays capturable)
        const int64_t m = (int64_t)a.n_showers * p.prof_bins;
        zero_kernel<<<64, 256, 0, st>>>(a.prof_ph, m);
        zero_kernel<<<64, 256, 0, st>>>(reinterpret_cast<double*>(a.prof_bu), m);
        if (int rc = check_launch("zero")) return rc;
    }
    if (p.params.event_begin) (void)hipEventRecord((hipEvent_t)p.params.event_begin, st);
    int rc = p.params.precision == 0
                 ? launch_emit_ts<0>(a, p.tile_segs, p.emit_grid, waves, lds, st)
                 : launch_emit_ts<1>(a, p.tile_segs, p.emit_grid, waves, lds, st);
    if (rc) return rc;
    if (p.params.event_end) (void)hipEventRecord((hipEvent_t)p.params.event_end, st);
    const int fin_grid = 1024;
    const size_t tel_lds = (size_t)a.n_tel * sizeof(int32_t);
    block_sum_kernel<<<fin_grid, 256, tel_lds, st>>>(a);
    if (int rc2 = check_launch("block_sum")) return rc2;
    cutoff_kernel<<<1, 1024, tel_lds, st>>>(a);
    if (int rc2 = check_launch("cutoff")) return rc2;
    rowblock_scan_kernel<<<fin_grid, 256, 0, st>>>(a);
    if (int rc2 = check_launch("rowblock_scan")) return rc2;
    if (a.n_tel <= kPrefixDenseTel) {
        tile_prefix_dense_kernel<<<fin_grid, 256, (size_t)kRowBlock * a.n_tel * sizeof(int32_t), st>>>(a);
    } else {
        const size_t prefix_lds = (size_t)((a.n_tel + 1) & ~1) * sizeof(int32_t) +
                                  (size_t)kPrefixLdsRuns * sizeof(int64_t);
        tile_prefix_kernel<<<fin_grid, kWave, prefix_lds, st>>>(a);
    }
    if (int rc2 = check_launch("tile_prefix")) return rc2;
    csr_kernel<<<1, 1024, 0, st>>>(a);
    if (int rc2 = check_launch("csr")) return rc2;
    scatter_kernel<<<4096, 256, 0, st>>>(a);
    return check_launch("scatter");
}

int launch_soft(RunPlan& p, const SoftPlan& sp, int mode)
{
    Args a = make_args(p);
    a.tile_segs = kSoftTS;          // the soft kernels walk 32-step tiles
    hipStream_t st = p.stream;
    const ckv_array* ar = p.arr;
    // the per-step cull's bound constants (screen_annulus), for the screening pass and
    // the FP64 tile kernels
    {
        const ckv_atmo* at = p.atmo;
        if (ar->screen_rmax > 0.0 && 1.0 + at->psi_min >= 0.5) {
            a.cull_rmax = ar->screen_rmax;
            a.cull_x0 = (at->psi_max - at->psi_min) / (1.0 + at->psi_min);
            a.cull_b0 = (at->psi_falls ? 0.5 : 0.8) * a.cull_x0;
            a.cull_rho2 = at->psi_falls ? 1.0 : (1.0 + at->psi_max) / (1.0 + at->psi_min);
        }
    }
    SoftArgs s{};
    s.nb_frozen = sp.n_b_frozen;
    s.sigma = sp.sigma;
    s.gS = sp.gS;
    s.gA = sp.gA;
    s.S = sp.S;
    s.A = sp.A;
    s.g_psi = sp.g_psi;
    s.g_P = sp.g_P;
    s.gx0 = ar->soft.gx0;
    s.gy0 = ar->soft.gy0;
    s.inv_cell = ar->soft.inv_cell;
    s.nx = ar->soft.nx;
    s.ny = ar->soft.ny;
    s.level_cells = ar->soft.level_cells;
    s.cell_off = ar->soft.d_cell_off;
    s.cell_list = ar->soft.d_cell_list;
    s.cell_ent = reinterpret_cast<const uint2*>(ar->soft.d_cell_ent);
    s.ids = sp.ids;
    s.ids_cap = sp.ids_cap;
    s.ids_count = sp.ids_count;
    // listed adjoint: bins, spheres and the lowest node records in LDS (at most
    // 128 KB for CKV_MAX_TEL spheres); beyond the LDS the adjoint recomputes everything
    size_t lds_l = (size_t)6 * soft_bin_nodes(a.n_nodes) * sizeof(double) +
                   (size_t)a.n_tel * 4 * sizeof(double) +
                   (size_t)kNode64 * soft_node_lds(a.n_nodes) * sizeof(double);
    if (mode == 1 && lds_l > 160 * 1024) s.ids_count = nullptr;
    // the listed kernels keep the per-shower table in LDS when it fits beside the rest
    const size_t shr_b = (size_t)a.n_showers * sizeof(ShowerRec);
    s.skip_if_listed = s.ids_count ? 1 : 0;
    // forward with a list: the screening pass (mixed bunch kernel against spheres of
    // the cut radius plus a margin, frozen counts) lists the candidates, FP64
    // recomputes them (soft_cand_kernel); the FP64 tile forward runs only if the
    // list overflowed
    Args e = a;
    int e_waves = 0;
    size_t e_lds = 0;
    if (mode == 0 && s.ids_count) {
        e.tel = ar->d_tel_screen;
        e.gx0 = ar->soft.gx0;
        e.gy0 = ar->soft.gy0;
        e.inv_cell = ar->soft.inv_cell;
        e.nx = ar->soft.nx;
        e.ny = ar->soft.ny;
        e.level_cells = ar->soft.level_cells;
        e.cell_off = ar->soft.d_cell_off;
        e.cell_list = ar->soft.d_cell_list;
        e.cell_ent = reinterpret_cast<const uint2*>(ar->soft.d_cell_ent);
        e.lds_entries = lds_entries(1, e.n_nodes, true);
        e.nb_frozen = sp.n_b_frozen;
        e.list_ids = sp.ids;
        e.list_cap = sp.ids_cap;
        e.list_count = sp.ids_count;
        const size_t tab = (table_bytes(1, e.n_nodes, true) + 15) & ~(size_t)15;
        const size_t per = wave_bytes(1, kSoftTS, e.n_tel, 0) + kScreenWaveBytes;
        for (int wv = kMaxEmitWaves; wv >= 1 && !e_waves; wv /= 2)
            if (tab + tel_bytes(e.n_tel) + (size_t)wv * per <= 160 * 1024) {
                e_waves = wv;
                e_lds = tab + tel_bytes(e.n_tel) + (size_t)wv * per;
            }
        if (!e_waves || e.n_nodes - 1 < 2) {
            set_error("soft response: tables too large for the screening pass");
            return CKV_ERR_TABLE;
        }
    }
    // as many waves as the kernel's launch bounds allow and the LDS holds
    const int wmax = soft_max_waves(mode);
    int waves = p.emit_waves > 0 && p.emit_waves < wmax ? p.emit_waves : wmax;
    while (waves > 1 && soft_lds_bytes(mode, a.n_nodes, a.n_tel, waves) > 160 * 1024) waves >>= 1;
    const size_t lds = soft_lds_bytes(mode, a.n_nodes, a.n_tel, waves);
    if (lds > 160 * 1024) {
        set_error("soft response: telescope count too large for LDS");
        return CKV_ERR_TABLE;
    }
    init_kernel<<<1, 1024, 0, st>>>(a);
    if (int rc = check_launch("init")) return rc;
    const int64_t nst = (int64_t)a.n_showers * a.n_tel;
    if (mode == 0) {
        zero_kernel<<<64, 256, 0, st>>>(s.S, nst);
        zero_kernel<<<64, 256, 0, st>>>(s.A, nst);
        // the list count starts at zero (all-zero bits: 0.0 is integer 0)
        if (s.ids_count) zero_kernel<<<1, 64, 0, st>>>(reinterpret_cast<double*>(s.ids_count), 1);
    } else {
        zero_kernel<<<64, 256, 0, st>>>(s.g_psi, a.n_nodes);
        zero_kernel<<<64, 256, 0, st>>>(s.g_P, (int64_t)5 * a.n_nodes);
    }
    if (int rc = check_launch("zero")) return rc;
    if (p.params.event_begin) (void)hipEventRecord((hipEvent_t)p.params.event_begin, st);
    if (mode == 0) {
        allow_lds((const void*)soft_kernel<0>, 160 * 1024);
        if (s.ids_count) {
            allow_lds((const void*)emit_kernel<1, kSoftTS, kFeatScreen>, 160 * 1024);
            emit_kernel<1, kSoftTS, kFeatScreen><<<p.emit_grid, e_waves * kWave, e_lds, st>>>(e);
            if (int rc = check_launch("screen")) return rc;
            size_t lds_c = (size_t)a.n_tel * 4 * sizeof(double) +
                           (size_t)kNode64 * soft_node_lds(a.n_nodes) * sizeof(double);
            const size_t acc_b = (size_t)2 * a.n_showers * a.n_tel * sizeof(double);
            s.cand_lds_acc = lds_c + acc_b <= 160 * 1024 ? 1 : 0;
            if (s.cand_lds_acc) lds_c += acc_b;
            s.shower_lds = lds_c + shr_b <= 160 * 1024 ? 1 : 0;
            if (s.shower_lds) lds_c += shr_b;
            allow_lds((const void*)soft_cand_kernel, 160 * 1024);
            soft_cand_kernel<<<2 * p.emit_grid, kSoftCandThreads, lds_c, st>>>(a, s);
            if (int rc = check_launch("soft candidates")) return rc;
        }
        soft_kernel<0><<<p.emit_grid, waves * kWave, lds, st>>>(a, s);
    } else {
        allow_lds((const void*)soft_kernel<1>, 160 * 1024);
        soft_kernel<1><<<p.emit_grid, waves * kWave, lds, st>>>(a, s);
        if (s.ids_count) {
            if (int rc = check_launch("soft")) return rc;
            s.shower_lds = lds_l + shr_b <= 160 * 1024 ? 1 : 0;
            if (s.shower_lds) lds_l += shr_b;
            allow_lds((const void*)soft_list_kernel, 160 * 1024);
            soft_list_kernel<<<2 * p.emit_grid, kSoftListThreads, lds_l, st>>>(a, s);
        }
    }
    if (int rc = check_launch("soft")) return rc;
    if (p.params.event_end) (void)hipEventRecord((hipEvent_t)p.params.event_end, st);
    return CKV_OK;
}

int launch_count(const ckv_segments* segs, const ckv_params* prm, const ckv_atmo* atmo, double k_ft,
                 int64_t* n_b, hipStream_t stream)
{
    RunPlan p{};
    p.segs = *segs;
    p.params = *prm;
    p.atmo = atmo;
    p.arr = nullptr;
    p.k_ft = k_ft;
    p.tile_segs = 1;
    Args a = make_args(p);
    if (segs->n == 0) return CKV_OK;
    const int64_t blocks = std::min<int64_t>((segs->n + 255) / 256, 65536);
    count_kernel<<<(unsigned)blocks, 256, 0, stream>>>(a, n_b);
    return check_launch("count");
}

}  // namespace ckv
