// C ABI entry points: argument validation, handle construction, workspace
// layout and the launch of one run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "ckv_internal.h"

namespace ckv {

namespace {
thread_local std::string g_error;

int hip_fail(const char* what, hipError_t e)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return CKV_ERR_HIP;
}

int profile_bins(const ckv_atmo* atmo, double bin_gcm2, int32_t* n_bins)
{
    if (atmo->depth.empty()) { set_error("the atmosphere has no depth table"); return CKV_ERR_ARG; }
    if (!(bin_gcm2 > 0.0) || !std::isfinite(bin_gcm2)) {
        set_error("depth bin width must be > 0"); return CKV_ERR_ARG;
    }
    const double nb = std::floor(atmo->depth[0] * (1.0 / bin_gcm2)) + 1.0;
    if (!(nb <= (double)CKV_MAX_PROFILE_BINS)) {
        set_error("more than CKV_MAX_PROFILE_BINS depth bins"); return CKV_ERR_ARG;
    }
    *n_bins = (int32_t)nb;
    return CKV_OK;
}

int device_cu_count(int* n_cu)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    return e == hipSuccess ? CKV_OK : hip_fail("device query", e);
}

template <typename T>
int upload(const T* host, size_t count, T** dev)
{
    hipError_t e = hipMalloc((void**)dev, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail("hipMalloc", e);
    e = hipMemcpy(*dev, host, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail("hipMemcpy", e);
    return CKV_OK;
}

double frank_tamm_k(double lambda_min_nm, double lambda_max_nm)
{
    // photons per metre of track per unit sin^2(theta_c): 2 pi alpha (1/l1 - 1/l2)
    return 2.0 * kPi * kFineStructure * (1.0 / lambda_min_nm - 1.0 / lambda_max_nm) * 1e9;
}

int check_params(const ckv_params* p)
{
    if (!p) { set_error("params is NULL"); return CKV_ERR_ARG; }
    if (!(p->bunch_size > 0.0) || !std::isfinite(p->bunch_size)) {
        set_error("bunch_size must be > 0"); return CKV_ERR_ARG;
    }
    if (!(p->lambda_min_nm > 0.0) || !(p->lambda_max_nm > p->lambda_min_nm) ||
        !std::isfinite(p->lambda_max_nm)) {
        set_error("need 0 < lambda_min < lambda_max"); return CKV_ERR_ARG;
    }
    if (!(p->w_min >= 0.0) || !(p->w_min < 1.0)) { set_error("need 0 <= w_min < 1"); return CKV_ERR_ARG; }
    if (p->precision != CKV_FP64 && p->precision != CKV_MIXED) {
        set_error("unknown precision"); return CKV_ERR_ARG;
    }
    if (p->tile_segments != 0 && p->tile_segments != 8 && p->tile_segments != 16 &&
        p->tile_segments != 32 && p->tile_segments != 64) {
        set_error("tile_segments must be 0 (default), 8, 16, 32 or 64"); return CKV_ERR_ARG;
    }
    if (p->grid < 0) { set_error("grid must be >= 0"); return CKV_ERR_ARG; }
    if (p->waves_per_group != 0 && p->waves_per_group != 1 && p->waves_per_group != 2 &&
        p->waves_per_group != 4 && p->waves_per_group != 8 && p->waves_per_group != 16) {
        set_error("waves_per_group must be 0, 1, 2, 4, 8 or 16"); return CKV_ERR_ARG;
    }
    if (!(p->depth_bin_gcm2 >= 0.0) || !std::isfinite(p->depth_bin_gcm2)) {
        set_error("depth_bin_gcm2 must be >= 0"); return CKV_ERR_ARG;
    }
    if ((p->grazing_exact != 0 && p->grazing_exact != 1) || p->reserved != 0) {
        set_error("grazing_exact must be 0 or 1, reserved 0"); return CKV_ERR_ARG;
    }
    if (!(p->earth_radius_m >= 0.0) || !std::isfinite(p->earth_radius_m)) {
        set_error("earth_radius_m must be >= 0"); return CKV_ERR_ARG;
    }
    if (p->earth_radius_m > 0.0 &&
        ((p->tile_segments != 0 && p->tile_segments != 32) || p->depth_bin_gcm2 > 0.0 ||
         p->grazing_exact)) {
        set_error("the curved atmosphere runs with tile_segments 0 or 32, without profile or "
                  "grazing_exact (every bunch is traced exactly)");
        return CKV_ERR_ARG;
    }
    return CKV_OK;
}

int check_segments(const ckv_segments* s)
{
    if (!s) { set_error("segments is NULL"); return CKV_ERR_ARG; }
    if (s->n < 0) { set_error("segment count < 0"); return CKV_ERR_ARG; }
    if (s->n > 0 && (!s->x0 || !s->y0 || !s->h0 || !s->u || !s->v || !s->w || !s->length ||
                     !s->t0 || !s->energy || !s->ptype)) {
        set_error("a segment array is NULL"); return CKV_ERR_ARG;
    }
    if (s->n >= ((int64_t)1 << 40)) { set_error("too many segments"); return CKV_ERR_ARG; }
    return CKV_OK;
}

int current_device(int want)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    if (dev != want) { set_error("handle was created on another device"); return CKV_ERR_ARG; }
    return CKV_OK;
}

constexpr int kDefaultTileSegs = 32;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

size_t workspace_layout(int64_t n_segments, int32_t n_showers, int32_t n_tel, int64_t capacity,
                        const ckv_params* p, RunPlan* plan, void* base)
{
    const int ts = (p && p->tile_segments > 0) ? p->tile_segments : kDefaultTileSegs;
    const int64_t max_tiles = n_segments / ts + n_showers + 1;
    const int64_t max_blocks = max_tiles / kRowBlock + n_showers + 1;
    const int64_t grid = (p && p->grid > 0) ? p->grid : kMaxEmitGrid;
    const int64_t n_waves = grid * kMaxEmitWaves;
    // crossings fill blocks back to back; each wave leaves at most one partial block
    const int64_t slots_needed = capacity + (n_waves + 1) * kStageBlock;
    const int64_t stage_blocks = (slots_needed + kStageBlock - 1) / kStageBlock;
    // a run holds at least one staged crossing: as many run slots as staging slots,
    // plus each wave's partly used run block, never run out first (tiles finish out
    // of order, so a smaller run array could be filled by later tiles and cut the
    // written prefix short)
    const int64_t run_blocks = stage_blocks * kStageBlock / kRunBlock + n_waves + 2;
    const int64_t run_cap = run_blocks * kRunBlock;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    size_t o_ctrl = take(sizeof(int64_t) * kCtrlSlots);
    size_t o_res = take(sizeof(ckv_result));
    size_t o_tb = take(sizeof(int64_t) * (n_showers + 1));
    size_t o_bb = take(sizeof(int64_t) * (n_showers + 1));
    size_t o_sf = take(sizeof(int64_t) * n_showers);
    size_t o_roff = take(sizeof(int64_t) * (size_t)max_tiles);
    size_t o_rn = take(sizeof(int32_t) * (size_t)max_tiles);
    size_t o_th = take(sizeof(int32_t) * (size_t)max_tiles);
    size_t o_runs = take(sizeof(int64_t) * (size_t)run_cap);
    size_t o_bsum = take(sizeof(int32_t) * (size_t)max_blocks * n_tel);
    size_t o_bh = take(sizeof(int64_t) * (size_t)max_blocks);
    size_t o_st = take(sizeof(int32_t) * (size_t)n_showers * n_tel);
    size_t o_fill = take(sizeof(int32_t) * (size_t)stage_blocks);
    size_t o_stage = take(sizeof(StageEntry) * (size_t)stage_blocks * kStageBlock);
    if (plan) {
        char* b = (char*)base;
        plan->tile_segs = ts;
        plan->max_tiles = max_tiles;
        plan->max_row_blocks = max_blocks;
        plan->stage_slots = stage_blocks * kStageBlock;
        plan->run_cap = run_cap;
        plan->ctrl = (int64_t*)(b + o_ctrl);
        plan->ws_result = (ckv_result*)(b + o_res);
        plan->tiles_before = (int64_t*)(b + o_tb);
        plan->blocks_before = (int64_t*)(b + o_bb);
        plan->shower_first = (int64_t*)(b + o_sf);
        plan->tile_run_off = (int64_t*)(b + o_roff);
        plan->tile_run_n = (int32_t*)(b + o_rn);
        plan->tile_hits = (int32_t*)(b + o_th);
        plan->runs = (int64_t*)(b + o_runs);
        plan->block_sums = (int32_t*)(b + o_bsum);
        plan->block_hits = (int64_t*)(b + o_bh);
        plan->shower_tel = (int32_t*)(b + o_st);
        plan->stage_fill = (int32_t*)(b + o_fill);
        plan->stage = (StageEntry*)(b + o_stage);
    }
    return off;
}

}  // namespace ckv

using namespace ckv;

static int atmo_create(const double* alt_m, const double* eta, const double* depth, int64_t n,
                       double obs_level_m, double step_m, ckv_atmo** out);

extern "C" {

const char* ckv_last_error(void) { return g_error.c_str(); }

int ckv_version(void) { return CKV_VERSION; }

int ckv_atmo_create_with_depth(const double* alt_m, const double* eta, const double* depth_gcm2,
                               int64_t n, double obs_level_m, double step_m, ckv_atmo** out)
{
    if (!alt_m || !eta || !out) { set_error("NULL argument"); return CKV_ERR_ARG; }
    *out = nullptr;
    if (n < 2) { set_error("atmosphere needs at least 2 points"); return CKV_ERR_ARG; }
    if (!(step_m >= 0.0) || !std::isfinite(step_m)) { set_error("step must be >= 0"); return CKV_ERR_ARG; }
    if (!std::isfinite(obs_level_m)) { set_error("observation level not finite"); return CKV_ERR_ARG; }
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(alt_m[i]) || !std::isfinite(eta[i]) || eta[i] < 0.0) {
            set_error("atmosphere: non-finite altitude or eta < 0"); return CKV_ERR_TABLE;
        }
        if (i > 0 && !(alt_m[i] > alt_m[i - 1])) {
            set_error("atmosphere: altitudes must increase strictly"); return CKV_ERR_TABLE;
        }
        if (depth_gcm2 && (!std::isfinite(depth_gcm2[i]) || (i > 0 && depth_gcm2[i] > depth_gcm2[i - 1]))) {
            set_error("atmosphere: depth must be finite and non-increasing with altitude");
            return CKV_ERR_TABLE;
        }
    }
    return atmo_create(alt_m, eta, depth_gcm2, n, obs_level_m, step_m, out);
}

int ckv_atmo_create(const double* alt_m, const double* eta, int64_t n, double obs_level_m,
                    double step_m, ckv_atmo** out)
{
    return ckv_atmo_create_with_depth(alt_m, eta, nullptr, n, obs_level_m, step_m, out);
}

int ckv_atmo_create_nodes(const double* alt_m, const double* eta, int64_t n, double obs_level_m,
                          ckv_atmo** out)
{
    if (!alt_m || !eta || !out) { set_error("NULL argument"); return CKV_ERR_ARG; }
    *out = nullptr;
    if (n < 2 || n > CKV_MAX_NODE_TABLE) {
        set_error("node tables need 2 .. CKV_MAX_NODE_TABLE points"); return CKV_ERR_ARG;
    }
    if (!std::isfinite(obs_level_m)) { set_error("observation level not finite"); return CKV_ERR_ARG; }
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(alt_m[i]) || !std::isfinite(eta[i]) || eta[i] < 0.0) {
            set_error("atmosphere: non-finite altitude or eta < 0"); return CKV_ERR_TABLE;
        }
        if (i > 0 && !(alt_m[i] > alt_m[i - 1])) {
            set_error("atmosphere: altitudes must increase strictly"); return CKV_ERR_TABLE;
        }
    }
    return atmo_create(alt_m, eta, nullptr, n, obs_level_m, -1.0, out);
}

int ckv_atmo_nodes(const ckv_atmo* atmo, double* h_nodes)
{
    if (!atmo || !h_nodes) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if (atmo->h_nodes.empty()) {
        for (int64_t i = 0; i < atmo->n_nodes; ++i) h_nodes[i] = atmo->h_obs + (double)i * atmo->step;
    } else {
        std::memcpy(h_nodes, atmo->h_nodes.data(), sizeof(double) * atmo->h_nodes.size());
    }
    return CKV_OK;
}

int ckv_atmo_depth(const ckv_atmo* atmo, double* depth)
{
    if (!atmo || !depth) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if (atmo->depth.empty()) { set_error("the atmosphere has no depth table"); return CKV_ERR_ARG; }
    std::memcpy(depth, atmo->depth.data(), sizeof(double) * atmo->depth.size());
    return CKV_OK;
}

int ckv_profile_bins(const ckv_atmo* atmo, double bin_gcm2, int32_t* n_bins)
{
    if (!atmo || !n_bins) { set_error("NULL argument"); return CKV_ERR_ARG; }
    return profile_bins(atmo, bin_gcm2, n_bins);
}


int ckv_atmo_from_params(const ckv_atmo_param_spec* spec, const double* theta, ckv_atmo** out)
{
    if (!out) { set_error("NULL argument"); return CKV_ERR_ARG; }
    *out = nullptr;
    int rc = param_spec_check(spec, theta);
    if (rc) return rc;
    std::vector<double> alt, eta;
    param_profile(spec, theta, &alt, &eta);
    if (alt.size() < 2) { set_error("fewer than two nodes"); return CKV_ERR_ARG; }
    return atmo_create(alt.data(), eta.data(), nullptr, (int64_t)alt.size(), spec->obs_level_m,
                       spec->step_m, out);
}

int ckv_atmo_params_backward(const ckv_atmo_param_spec* spec, const double* theta,
                             const ckv_atmo* atmo, const double* g_psi, const double* g_P,
                             double* g_theta)
{
    int rc = param_spec_check(spec, theta);
    if (rc) return rc;
    if (!atmo || !g_psi || !g_P || !g_theta) { set_error("NULL argument"); return CKV_ERR_ARG; }
    param_backward(spec, theta, atmo, g_psi, g_P, g_theta);
    return CKV_OK;
}

int ckv_atmo_info(const ckv_atmo* a, int64_t* n_nodes, double* obs_level_m, double* step_m)
{
    if (!a) { set_error("NULL atmosphere"); return CKV_ERR_ARG; }
    if (n_nodes) *n_nodes = a->n_nodes;
    if (obs_level_m) *obs_level_m = a->h_obs;
    if (step_m) *step_m = a->step;
    return CKV_OK;
}

int ckv_atmo_tables(const ckv_atmo* a, double* psi, double* P)
{
    if (!a) { set_error("NULL atmosphere"); return CKV_ERR_ARG; }
    if (psi) std::memcpy(psi, a->psi.data(), sizeof(double) * a->psi.size());
    if (P) std::memcpy(P, a->P.data(), sizeof(double) * a->P.size());
    return CKV_OK;
}

int ckv_atmo_destroy(ckv_atmo* a)
{
    if (!a) return CKV_OK;
    if (a->d_node64) (void)hipFree(a->d_node64);
    if (a->d_cell32) (void)hipFree(a->d_cell32);
    if (a->d_depth) (void)hipFree(a->d_depth);
    if (a->d_hnodes) (void)hipFree(a->d_hnodes);
    delete a;
    return CKV_OK;
}

static int upload_grid(ckv_grid* g)
{
    int rc;
    if ((rc = upload(g->cell_off.data(), g->cell_off.size(), &g->d_cell_off)) ||
        (rc = upload(g->cell_list.data(), g->cell_list.size(), &g->d_cell_list)) ||
        (rc = upload(g->cell_ent.data(), g->cell_ent.size(), &g->d_cell_ent)))
        return rc;
    return CKV_OK;
}

static void free_grid(ckv_grid* g)
{
    if (g->d_cell_off) (void)hipFree(g->d_cell_off);
    if (g->d_cell_list) (void)hipFree(g->d_cell_list);
    if (g->d_cell_ent) (void)hipFree(g->d_cell_ent);
    g->d_cell_off = nullptr;
    g->d_cell_list = nullptr;
    g->d_cell_ent = nullptr;
}

static int array_create(const double* x_m, const double* y_m, const double* r_m, int32_t n_tel,
                        double sigma, ckv_array** out)
{
    if (!x_m || !y_m || !r_m || !out) { set_error("NULL argument"); return CKV_ERR_ARG; }
    *out = nullptr;
    if (n_tel < 1 || n_tel > CKV_MAX_TEL) { set_error("need 1 <= n_tel <= CKV_MAX_TEL"); return CKV_ERR_ARG; }
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) { set_error("sigma must be >= 0"); return CKV_ERR_ARG; }
    for (int32_t k = 0; k < n_tel; ++k)
        if (!std::isfinite(x_m[k]) || !std::isfinite(y_m[k]) || !std::isfinite(r_m[k]) || !(r_m[k] > 0.0)) {
            set_error("telescopes: non-finite position or radius <= 0"); return CKV_ERR_TABLE;
        }
    ckv_array* arr = new (std::nothrow) ckv_array();
    if (!arr) { set_error("out of host memory"); return CKV_ERR_NOMEM; }
    arr->n_tel = n_tel;
    arr->x.assign(x_m, x_m + n_tel);
    arr->y.assign(y_m, y_m + n_tel);
    arr->r.assign(r_m, r_m + n_tel);
    arr->soft_sigma = sigma;
    int rc = build_array_grid(arr, arr->r, &arr->hit);
    std::vector<double> tel_screen;
    if (!rc && sigma > 0.0) {
        // beyond sqrt(R^2 + 2 R sigma z_cut) the soft weight is exactly zero; the grid
        // and the screening spheres add a margin for the mixed-precision screening pass
        std::vector<double> reff(n_tel);
        tel_screen.resize(4 * (size_t)n_tel);
        for (int32_t k = 0; k < n_tel; ++k) {
            reff[k] = std::sqrt(r_m[k] * r_m[k] + 2.0 * r_m[k] * sigma * kSoftZCut) * (1.0 + 1e-9) +
                      kScreenMargin;
            tel_screen[4 * k] = x_m[k];
            tel_screen[4 * k + 1] = y_m[k];
            tel_screen[4 * k + 2] = reff[k];
            tel_screen[4 * k + 3] = reff[k] * reff[k];
            arr->screen_rmax = std::max(arr->screen_rmax, reff[k]);
        }
        rc = build_array_grid(arr, reff, &arr->soft);
    }
    if (!rc) {
        const hipError_t e = hipGetDevice(&arr->device);
        if (e != hipSuccess) rc = hip_fail("hipGetDevice", e);
    }
    if (rc) { ckv_array_destroy(arr); return rc; }
    std::vector<double> tel(4 * (size_t)n_tel);
    for (int32_t k = 0; k < n_tel; ++k) {
        tel[4 * k] = x_m[k];
        tel[4 * k + 1] = y_m[k];
        tel[4 * k + 2] = r_m[k];
        tel[4 * k + 3] = r_m[k] * r_m[k];
    }
    if ((rc = upload(tel.data(), tel.size(), &arr->d_tel)) || (rc = upload_grid(&arr->hit)) ||
        (sigma > 0.0 && (rc = upload_grid(&arr->soft))) ||
        (sigma > 0.0 && (rc = upload(tel_screen.data(), tel_screen.size(), &arr->d_tel_screen)))) {
        ckv_array_destroy(arr);
        return rc;
    }
    *out = arr;
    return CKV_OK;
}

int ckv_array_create(const double* x_m, const double* y_m, const double* r_m, int32_t n_tel,
                     ckv_array** out)
{
    return array_create(x_m, y_m, r_m, n_tel, 0.0, out);
}

int ckv_array_create_soft(const double* x_m, const double* y_m, const double* r_m, int32_t n_tel,
                          double sigma_m, ckv_array** out)
{
    if (!(sigma_m > 0.0)) { set_error("sigma must be > 0"); return CKV_ERR_ARG; }
    return array_create(x_m, y_m, r_m, n_tel, sigma_m, out);
}

int ckv_array_destroy(ckv_array* arr)
{
    if (!arr) return CKV_OK;
    if (arr->d_tel) (void)hipFree(arr->d_tel);
    if (arr->d_tel_screen) (void)hipFree(arr->d_tel_screen);
    free_grid(&arr->hit);
    free_grid(&arr->soft);
    delete arr;
    return CKV_OK;
}

size_t ckv_workspace_size(int64_t n_segments, int32_t n_showers, int32_t n_tel, int64_t capacity,
                          const ckv_params* params)
{
    if (n_segments < 0 || n_showers < 1 || n_tel < 1 || capacity < 0) return 0;
    return workspace_layout(n_segments, n_showers, n_tel, capacity, params, nullptr, nullptr);
}

int ckv_run(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
            const ckv_atmo* atmo, const ckv_array* arr, void* workspace, size_t ws_bytes,
            ckv_output* out, const ckv_cursor* resume_from, void* stream)
{
    return run_checked(segs, showers, params, atmo, arr, workspace, ws_bytes, out, resume_from,
                       stream);
}

}  // extern "C"

namespace ckv {

int run_checked(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                const ckv_atmo* atmo, const ckv_array* arr, void* workspace, size_t ws_bytes,
                ckv_output* out, const ckv_cursor* resume_from, void* stream)
{
    int rc;
    if ((rc = check_segments(segs)) || (rc = check_params(params))) return rc;
    if (!showers || !atmo || !arr || !out || !workspace) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if (showers->n_showers < 1 || !showers->seg_offsets || !showers->t_ref) {
        set_error("showers: need n_showers >= 1, seg_offsets and t_ref"); return CKV_ERR_ARG;
    }
    if (!out->tel_offsets || !out->result || out->capacity < 0 || (out->capacity > 0 && !out->records)) {
        set_error("output: tel_offsets, result and records (capacity > 0) are required");
        return CKV_ERR_ARG;
    }
    if (!atmo->h_nodes.empty() &&
        ((params->tile_segments != 0 && params->tile_segments != 32) || params->depth_bin_gcm2 > 0.0 ||
         params->grazing_exact || params->earth_radius_m > 0.0)) {
        set_error("node tables run with tile_segments 0 or 32, without profile, exact grazing "
                  "path or curved atmosphere");
        return CKV_ERR_ARG;
    }
    int32_t prof_bins = 0;
    if (params->depth_bin_gcm2 > 0.0) {
        if ((rc = profile_bins(atmo, params->depth_bin_gcm2, &prof_bins))) return rc;
        if (!out->profile_photons || !out->profile_bunches) {
            set_error("output: profile_photons and profile_bunches are required for a profile");
            return CKV_ERR_ARG;
        }
    }
    if (resume_from && (resume_from->step < 0 || resume_from->step > segs->n ||
                        resume_from->shower < 0 || resume_from->shower >= showers->n_showers ||
                        resume_from->reserved != 0)) {
        set_error("resume cursor: need 0 <= step <= n, 0 <= shower < n_showers, reserved 0");
        return CKV_ERR_ARG;
    }
    if ((rc = current_device(atmo->device)) || (rc = current_device(arr->device))) return rc;
    RunPlan plan{};
    plan.prof_bins = prof_bins;
    plan.cursor = resume_from ? *resume_from : ckv_cursor{0, 0, 0};
    size_t need = workspace_layout(segs->n, showers->n_showers, arr->n_tel, out->capacity, params,
                                   &plan, workspace);
    if (ws_bytes < need) {
        set_error("workspace smaller than ckv_workspace_size()"); return CKV_ERR_CAPACITY;
    }
    plan.segs = *segs;
    plan.showers = *showers;
    plan.params = *params;
    plan.atmo = atmo;
    plan.arr = arr;
    plan.out = *out;
    plan.stream = (hipStream_t)stream;
    plan.k_ft = frank_tamm_k(params->lambda_min_nm, params->lambda_max_nm);
    int n_cu = 256;
    if (int rc = device_cu_count(&n_cu)) return rc;
    plan.emit_grid = params->grid > 0 ? params->grid : std::min(n_cu, kMaxEmitGrid);
    // default: 16 waves for the mixed kernel, 8 for FP64 (16 is its narrow build)
    plan.emit_waves = params->waves_per_group > 0 ? params->waves_per_group
                      : params->precision == CKV_FP64 ? kMaxEmitWaves / 2 : kMaxEmitWaves;
    return launch_run(plan);
}

int default_emit_grid(int* grid)
{
    int n_cu = 256;
    if (int rc = device_cu_count(&n_cu)) return rc;
    *grid = std::min(n_cu, kMaxEmitGrid);
    return CKV_OK;
}

}  // namespace ckv

extern "C" {

static int soft_common(const ckv_segments* segs, const ckv_showers* showers,
                       const ckv_params* params, const ckv_atmo* atmo, const ckv_array* arr,
                       const int64_t* n_b_frozen, ckv_result* result, void* workspace,
                       size_t ws_bytes, void* stream, RunPlan* plan)
{
    int rc;
    if ((rc = check_segments(segs)) || (rc = check_params(params))) return rc;
    if (!showers || !atmo || !arr || !workspace || (!n_b_frozen && segs->n > 0)) {
        set_error("NULL argument"); return CKV_ERR_ARG;
    }
    if (showers->n_showers < 1 || !showers->seg_offsets || !showers->t_ref) {
        set_error("showers: need n_showers >= 1, seg_offsets and t_ref"); return CKV_ERR_ARG;
    }
    if (!(arr->soft_sigma > 0.0)) {
        set_error("telescope handle has no soft grid (use ckv_array_create_soft)"); return CKV_ERR_ARG;
    }
    if (!atmo->h_nodes.empty()) {
        set_error("the soft response needs a uniform-grid atmosphere"); return CKV_ERR_ARG;
    }
    if (params->earth_radius_m > 0.0) {
        set_error("the soft response is defined for the plane-parallel atmosphere"); return CKV_ERR_ARG;
    }
    if ((rc = current_device(atmo->device)) || (rc = current_device(arr->device))) return rc;
    size_t need = workspace_layout(segs->n, showers->n_showers, arr->n_tel, 0, params, plan, workspace);
    if (ws_bytes < need) { set_error("workspace smaller than ckv_workspace_size()"); return CKV_ERR_CAPACITY; }
    plan->segs = *segs;
    plan->showers = *showers;
    plan->params = *params;
    plan->atmo = atmo;
    plan->arr = arr;
    plan->stream = (hipStream_t)stream;
    // device-side conditions go to the caller's report, else to the workspace's own
    plan->out.result = result ? result : plan->ws_result;
    plan->k_ft = frank_tamm_k(params->lambda_min_nm, params->lambda_max_nm);
    int n_cu = 256;
    if (int rc = device_cu_count(&n_cu)) return rc;
    plan->emit_grid = params->grid > 0 ? params->grid : std::min(n_cu, kMaxEmitGrid);
    plan->emit_waves = 0;            // as many as the LDS holds
    return CKV_OK;
}

static int check_list(const ckv_soft_list* list)
{
    if (list && (list->capacity < 0 || !list->count || (list->capacity > 0 && !list->ids))) {
        set_error("soft list: need capacity >= 0, count and (capacity > 0) ids");
        return CKV_ERR_ARG;
    }
    return CKV_OK;
}

int ckv_soft_forward(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                     const ckv_atmo* atmo, const ckv_array* arr, const int64_t* n_b_frozen,
                     double* S, double* A, const ckv_soft_list* list, ckv_result* result,
                     void* workspace, size_t ws_bytes, void* stream)
{
    RunPlan plan{};
    if (int rc = soft_common(segs, showers, params, atmo, arr, n_b_frozen, result, workspace,
                             ws_bytes, stream, &plan))
        return rc;
    if (!S || !A) { set_error("NULL output"); return CKV_ERR_ARG; }
    if (int rc = check_list(list)) return rc;
    SoftPlan sp{};
    if (list) {
        sp.ids = list->ids;
        sp.ids_cap = list->capacity;
        sp.ids_count = list->count;
    }
    sp.n_b_frozen = n_b_frozen;
    sp.sigma = arr->soft_sigma;
    sp.S = S;
    sp.A = A;
    return launch_soft(plan, sp, 0);
}

int ckv_soft_backward(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                      const ckv_atmo* atmo, const ckv_array* arr, const int64_t* n_b_frozen,
                      const double* dL_dS, const double* dL_dA, double* g_psi, double* g_P,
                      const ckv_soft_list* list, ckv_result* result, void* workspace,
                      size_t ws_bytes, void* stream)
{
    RunPlan plan{};
    if (int rc = soft_common(segs, showers, params, atmo, arr, n_b_frozen, result, workspace,
                             ws_bytes, stream, &plan))
        return rc;
    if (!dL_dS || !dL_dA || !g_psi || !g_P) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if (int rc = check_list(list)) return rc;
    SoftPlan sp{};
    if (list) {
        sp.ids = list->ids;
        sp.ids_cap = list->capacity;
        sp.ids_count = list->count;
    }
    sp.n_b_frozen = n_b_frozen;
    sp.sigma = arr->soft_sigma;
    sp.gS = dL_dS;
    sp.gA = dL_dA;
    sp.g_psi = g_psi;
    sp.g_P = g_P;
    return launch_soft(plan, sp, 1);
}

int ckv_count(const ckv_segments* segs, const ckv_params* params, const ckv_atmo* atmo,
              int64_t* n_b, void* stream)
{
    int rc;
    if ((rc = check_segments(segs)) || (rc = check_params(params))) return rc;
    if (!atmo || (!n_b && segs->n > 0)) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if ((rc = current_device(atmo->device))) return rc;
    return launch_count(segs, params, atmo, frank_tamm_k(params->lambda_min_nm, params->lambda_max_nm),
                        n_b, (hipStream_t)stream);
}

}  // extern "C"

static int atmo_create(const double* alt_m, const double* eta, const double* depth, int64_t n,
                       double obs_level_m, double step_m, ckv_atmo** out)
{
    ckv_atmo* a = new (std::nothrow) ckv_atmo();
    if (!a) { set_error("out of host memory"); return CKV_ERR_NOMEM; }
    // step_m < 0 asks for node tables on the input's own altitudes
    int rc = step_m < 0.0 ? build_node_tables(alt_m, eta, n, obs_level_m, a)
                          : build_atmo_tables(alt_m, eta, n, obs_level_m, step_m, a);
    if (rc) { delete a; return rc; }
    if (depth) build_depth_table(alt_m, depth, n, a);
    if (a->n_nodes > (1 << 20)) { delete a; set_error("atmosphere table too fine"); return CKV_ERR_TABLE; }
    {
        const hipError_t e = hipGetDevice(&a->device);
        if (e != hipSuccess) { delete a; return hip_fail("hipGetDevice", e); }
    }
    const int64_t m = a->n_nodes;
    std::vector<double> node(m * kNode64);
    for (int64_t i = 0; i < m; ++i) {
        node[i * kNode64] = a->psi[i];
        for (int j = 0; j < 5; ++j) node[i * kNode64 + 1 + j] = a->P[j * m + i];
    }
    std::vector<float> cell((m - 1) * kCell32, 0.0f);
    for (int64_t i = 0; i + 1 < m; ++i) {
        float* c = &cell[i * kCell32];
        c[0] = (float)a->psi[i];
        c[1] = (float)(a->psi[i + 1] - a->psi[i]);
        for (int j = 0; j < 5; ++j) c[2 + j] = (float)a->P[j * m + i];
        // node height above the observation level
        c[7] = (float)(a->h_nodes.empty() ? (double)i * a->step : a->h_nodes[i] - a->h_obs);
    }
    std::vector<double> hinfo;   // node tables: altitudes, then inverse cell widths
    if (!a->h_nodes.empty()) {
        hinfo = a->h_nodes;
        for (int64_t i = 0; i + 1 < m; ++i) hinfo.push_back(1.0 / (a->h_nodes[i + 1] - a->h_nodes[i]));
    }
    if ((rc = upload(node.data(), node.size(), &a->d_node64)) ||
        (rc = upload(cell.data(), cell.size(), &a->d_cell32)) ||
        (!a->depth.empty() && (rc = upload(a->depth.data(), a->depth.size(), &a->d_depth))) ||
        (!hinfo.empty() && (rc = upload(hinfo.data(), hinfo.size(), &a->d_hnodes)))) {
        ckv_atmo_destroy(a);
        return rc;
    }
    *out = a;
    return CKV_OK;
}
