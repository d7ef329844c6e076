// Host-side construction of the atmosphere tables and the telescope candidate
// grid.  Both are built once per handle (sec. 3.3.2: fine uniform tables are
// computed at initialisation so that lookups need no search).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ckv_internal.h"

namespace ckv {

namespace {

// n-1 at altitude h, linear between the bracketing input points (sec. 3.3.1);
// an input point is returned exactly.
double profile_at(const double* alt, const double* eta, int64_t n, double h)
{
#pragma clang fp contract(off)
    const double* it = std::upper_bound(alt, alt + n, h);   // first alt > h
    int64_t hi = it - alt;
    int64_t lo = hi - 1;
    if (lo >= 0 && alt[lo] == h) return eta[lo];
    if (hi >= n) return eta[n - 1];
    if (lo < 0) return eta[0];
    double f = (h - alt[lo]) / (alt[hi] - alt[lo]);
    return eta[lo] + f * (eta[hi] - eta[lo]);
}

}  // namespace

int build_atmo_tables(const double* alt, const double* eta, int64_t n, double h_obs, double step,
                      ckv_atmo* a)
{
#pragma clang fp contract(off)
    if (!(step > 0.0)) step = alt[1] - alt[0];
    if (!(step > 0.0)) {
        set_error("atmosphere: non-positive altitude step");
        return CKV_ERR_TABLE;
    }
    if (!(h_obs >= alt[0]) || !(h_obs < alt[n - 1])) {
        set_error("atmosphere: observation level outside the profile");
        return CKV_ERR_TABLE;
    }
    // nodes h_obs + i*step inside the profile
    int64_t m = (int64_t)std::floor((alt[n - 1] - h_obs) / step) + 1;
    while (m > 1 && h_obs + (double)(m - 1) * step > alt[n - 1]) --m;
    if (m < 2) {
        set_error("atmosphere: fewer than two table nodes above the observation level");
        return CKV_ERR_TABLE;
    }
    a->n_nodes = m;
    a->h_obs = h_obs;
    a->step = step;
    a->inv_step = 1.0 / step;
    a->h_top = h_obs + (double)(m - 1) * step;
    a->psi.assign(m, 0.0);
    a->P.assign(5 * m, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        double e = profile_at(alt, eta, n, h_obs + (double)i * step);
        a->psi[i] = e * (2.0 + e);                  // n^2 - 1
    }
    // P_j(h_{i+1}) = P_j(h_i) + step/(j+1) * sum_{m=0..j} psi_i^(j-m) psi_{i+1}^m,
    // the exact cell integral of psi^j for psi linear in the cell
    for (int64_t i = 0; i + 1 < m; ++i) {
        double lo = a->psi[i], hi = a->psi[i + 1];
        double hs = 1.0, hp = 1.0;   // complete homogeneous sums h_j(lo, hi), powers of hi
        for (int j = 1; j <= 5; ++j) {
            hp = hp * hi;
            hs = lo * hs + hp;
            a->P[(j - 1) * m + i + 1] = a->P[(j - 1) * m + i] + step * hs / (double)(j + 1);
        }
    }
    a->n_obs = std::sqrt(1.0 + a->psi[0]);
    psi_range(a);
    return CKV_OK;
}

void psi_range(ckv_atmo* a)
{
    a->psi_min = a->psi_max = a->psi[0];
    a->psi_falls = true;
    for (size_t i = 1; i < a->psi.size(); ++i) {
        a->psi_min = std::min(a->psi_min, a->psi[i]);
        a->psi_max = std::max(a->psi_max, a->psi[i]);
        if (!(a->psi[i] <= a->psi[i - 1])) a->psi_falls = false;
    }
}

int build_node_tables(const double* alt, const double* eta, int64_t n, double h_obs, ckv_atmo* a)
{
#pragma clang fp contract(off)
    if (!(h_obs >= alt[0]) || !(h_obs < alt[n - 1])) {
        set_error("atmosphere: observation level outside the profile");
        return CKV_ERR_TABLE;
    }
    a->h_nodes.clear();
    a->h_nodes.push_back(h_obs);
    for (int64_t i = 0; i < n; ++i)
        if (alt[i] > h_obs) a->h_nodes.push_back(alt[i]);
    const int64_t m = (int64_t)a->h_nodes.size();
    a->n_nodes = m;
    a->h_obs = h_obs;
    a->step = 0.0;               // not a uniform grid
    a->inv_step = 0.0;
    a->h_top = a->h_nodes[m - 1];
    a->psi.assign(m, 0.0);
    a->P.assign(5 * m, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        double e = profile_at(alt, eta, n, a->h_nodes[i]);
        a->psi[i] = e * (2.0 + e);
    }
    // the cell integral of psi^j for psi linear over a cell of width h_{i+1} - h_i
    for (int64_t i = 0; i + 1 < m; ++i) {
        double lo = a->psi[i], hi = a->psi[i + 1], width = a->h_nodes[i + 1] - a->h_nodes[i];
        double hs = 1.0, hp = 1.0;
        for (int j = 1; j <= 5; ++j) {
            hp = hp * hi;
            hs = lo * hs + hp;
            a->P[(j - 1) * m + i + 1] = a->P[(j - 1) * m + i] + width * hs / (double)(j + 1);
        }
    }
    a->n_obs = std::sqrt(1.0 + a->psi[0]);
    psi_range(a);
    return CKV_OK;
}

void build_depth_table(const double* alt, const double* depth, int64_t n, ckv_atmo* a)
{
#pragma clang fp contract(off)
    a->depth.assign(a->n_nodes, 0.0);
    for (int64_t i = 0; i < a->n_nodes; ++i)
        a->depth[i] = profile_at(alt, depth, n, a->h_obs + (double)i * a->step);
}

int build_array_grid(const ckv_array* arr, const std::vector<double>& radius, ckv_grid* g)
{
    const int32_t n = arr->n_tel;
    double rmax = 0, xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int32_t k = 0; k < n; ++k) {
        double reach = radius[k] / kGridWLevel[0];
        rmax = std::max(rmax, radius[k]);
        xmin = std::min(xmin, arr->x[k] - reach);
        xmax = std::max(xmax, arr->x[k] + reach);
        ymin = std::min(ymin, arr->y[k] - reach);
        ymax = std::max(ymax, arr->y[k] + reach);
    }
    double extent = std::max(xmax - xmin, ymax - ymin);
    double margin = 0.01 + 1e-9 * extent;
    double cell = std::max(rmax, extent / 512.0);
    xmin -= margin; ymin -= margin;
    int32_t nx = (int32_t)std::ceil((xmax + margin - xmin) / cell) + 1;
    int32_t ny = (int32_t)std::ceil((ymax + margin - ymin) / cell) + 1;
    g->gx0 = xmin;
    g->gy0 = ymin;
    g->cell = cell;
    g->inv_cell = 1.0 / cell;
    g->nx = nx;
    g->ny = ny;
    g->level_cells = nx * ny;
    const size_t n_cells = (size_t)nx * ny;
    g->cell_off.assign(kGridLevels * n_cells + 1, 0);
    std::vector<std::vector<uint16_t>> lists(kGridLevels * n_cells);
    for (int lv = 0; lv < kGridLevels; ++lv)
        for (int32_t k = 0; k < n; ++k) {
            double reach = radius[k] / kGridWLevel[lv] + margin;
            int32_t ix0 = std::max(0, (int32_t)std::floor((arr->x[k] - reach - xmin) / cell));
            int32_t ix1 = std::min(nx - 1, (int32_t)std::floor((arr->x[k] + reach - xmin) / cell));
            int32_t iy0 = std::max(0, (int32_t)std::floor((arr->y[k] - reach - ymin) / cell));
            int32_t iy1 = std::min(ny - 1, (int32_t)std::floor((arr->y[k] + reach - ymin) / cell));
            for (int32_t ix = ix0; ix <= ix1; ++ix)
                for (int32_t iy = iy0; iy <= iy1; ++iy) {
                    // distance from the centre to the cell rectangle
                    double cx0 = xmin + ix * cell, cy0 = ymin + iy * cell;
                    double dx = std::max({cx0 - arr->x[k], 0.0, arr->x[k] - (cx0 + cell)});
                    double dy = std::max({cy0 - arr->y[k], 0.0, arr->y[k] - (cy0 + cell)});
                    if (dx * dx + dy * dy <= reach * reach)
                        lists[lv * n_cells + (size_t)ix * ny + iy].push_back((uint16_t)k);
                }
        }
    g->cell_list.clear();
    for (size_t c = 0; c < lists.size(); ++c) {
        g->cell_off[c] = (int32_t)g->cell_list.size();
        g->cell_list.insert(g->cell_list.end(), lists[c].begin(), lists[c].end());
    }
    g->cell_off[lists.size()] = (int32_t)g->cell_list.size();
    g->cell_ent.assign(2 * lists.size(), 0u);
    for (size_t c = 0; c < lists.size(); ++c) {
        const uint32_t cnt = (uint32_t)lists[c].size();
        g->cell_ent[2 * c] = (uint32_t)g->cell_off[c];
        g->cell_ent[2 * c + 1] = cnt | ((cnt ? (uint32_t)lists[c][0] : 0u) << 16);
    }
    if (g->cell_list.empty()) g->cell_list.push_back(0);
    return CKV_OK;
}

// ---------------------------------------------------------------------------
// Parameterised atmosphere (differentiation pattern):
//   log eta(h) = log eta0 - sum_l overlap([0, h], layer l) / H_l + Lambda(h),
// Lambda the linear interpolant of knot values at h_j = j*knot_top/(n_knots-1),
// constant above knot_top; the last layer extends upward.
// ---------------------------------------------------------------------------
namespace {

struct KnotPos {
    int32_t j;
    double f;
};

KnotPos knot_pos(const ckv_atmo_param_spec* sp, double h)
{
#pragma clang fp contract(off)
    double hc = h < sp->knot_top_m ? h : sp->knot_top_m;
    double dk = sp->knot_top_m / (double)(sp->n_knots - 1);
    double x = hc / dk;
    int32_t j = (int32_t)std::floor(x);
    if (j > sp->n_knots - 2) j = sp->n_knots - 2;
    if (j < 0) j = 0;
    return {j, x - (double)j};
}

double layer_overlap(const ckv_atmo_param_spec* sp, int32_t l, double h)
{
#pragma clang fp contract(off)
    double top = (l + 1 < sp->n_layers) ? sp->layer_bounds_m[l + 1] : INFINITY;
    double hi = h < top ? h : top;
    double over = hi - sp->layer_bounds_m[l];
    return over > 0.0 ? over : 0.0;
}

double log_eta_param(const ckv_atmo_param_spec* sp, const double* theta, double h)
{
#pragma clang fp contract(off)
    const double* knots = theta;
    const double* H = theta + sp->n_knots;
    double depth = 0.0;
    for (int32_t l = 0; l < sp->n_layers; ++l) {
        double over = layer_overlap(sp, l, h);
        if (over > 0.0) depth += over / H[l];
    }
    KnotPos kp = knot_pos(sp, h);
    double lam = knots[kp.j] + kp.f * (knots[kp.j + 1] - knots[kp.j]);
    return std::log(sp->eta0) - depth + lam;
}

}  // namespace

int param_spec_check(const ckv_atmo_param_spec* sp, const double* theta)
{
    if (!sp || !theta || !sp->layer_bounds_m) { set_error("NULL argument"); return CKV_ERR_ARG; }
    if (sp->n_layers < 1 || sp->n_layers > 64 || sp->n_knots < 2 || sp->n_knots > 4096) {
        set_error("need 1 <= n_layers <= 64 and 2 <= n_knots <= 4096"); return CKV_ERR_ARG;
    }
    if (!(sp->eta0 > 0.0) || !(sp->knot_top_m > 0.0) || !(sp->step_m > 0.0) ||
        !(sp->top_m > sp->obs_level_m) || !(sp->obs_level_m >= sp->layer_bounds_m[0])) {
        set_error("parameterised atmosphere: bad eta0, knot_top, step or altitude range");
        return CKV_ERR_ARG;
    }
    for (int32_t l = 0; l < sp->n_layers; ++l) {
        if (!(sp->layer_bounds_m[l + 1] > sp->layer_bounds_m[l])) {
            set_error("layer bounds must increase"); return CKV_ERR_ARG;
        }
        if (!(theta[sp->n_knots + l] > 0.0)) { set_error("scale heights must be > 0"); return CKV_ERR_ARG; }
    }
    for (int32_t j = 0; j < sp->n_knots + sp->n_layers; ++j)
        if (!std::isfinite(theta[j])) { set_error("non-finite parameter"); return CKV_ERR_ARG; }
    return CKV_OK;
}

void param_profile(const ckv_atmo_param_spec* sp, const double* theta, std::vector<double>* alt,
                   std::vector<double>* eta)
{
    int64_t m = (int64_t)std::floor((sp->top_m - sp->obs_level_m) / sp->step_m) + 1;
    alt->resize(m);
    eta->resize(m);
    for (int64_t i = 0; i < m; ++i) {
        double h = sp->obs_level_m + (double)i * sp->step_m;
        (*alt)[i] = h;
        (*eta)[i] = std::exp(log_eta_param(sp, theta, h));
    }
}

// Reverse of theta -> eta_i -> psi_i -> P_j(h_i):
//   P_j(h_i) = sum_{m<i} c_j(psi_m, psi_{m+1}),  c_j(a, b) = step/(j+1) h_j(a, b),
// so dL/dpsi_m collects suffix sums of dL/dP_j over the nodes above m.
void param_backward(const ckv_atmo_param_spec* sp, const double* theta, const ckv_atmo* a,
                    const double* g_psi, const double* g_P, double* g_theta)
{
    const int64_t m = a->n_nodes;
    const double step = a->step;
    std::vector<double> gpsi(g_psi, g_psi + m);
    double suffix[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // per j: sum of g_P_j over nodes >= c + 1
    for (int64_t c = m - 2; c >= 0; --c) {
        const double lo = a->psi[c], hi = a->psi[c + 1];
        double pl[5], ph[5];                       // lo^k, hi^k for k < 5
        pl[0] = ph[0] = 1.0;
        for (int k = 1; k < 5; ++k) {
            pl[k] = pl[k - 1] * lo;
            ph[k] = ph[k - 1] * hi;
        }
        for (int j = 1; j <= 5; ++j) {
            suffix[j] += g_P[(size_t)(j - 1) * m + c + 1];
            // d h_j / d lo and d h_j / d hi, h_j(lo, hi) = sum_q lo^(j-q) hi^q
            double dlo = 0.0, dhi = 0.0;
            for (int q = 0; q < j; ++q) dlo += (double)(j - q) * pl[j - q - 1] * ph[q];
            for (int q = 1; q <= j; ++q) dhi += (double)q * pl[j - q] * ph[q - 1];
            const double w = step / (double)(j + 1);
            gpsi[c] += suffix[j] * w * dlo;
            gpsi[c + 1] += suffix[j] * w * dhi;
        }
    }
    const int32_t nk = sp->n_knots, nl = sp->n_layers;
    for (int32_t q = 0; q < nk + nl; ++q) g_theta[q] = 0.0;
    const double* H = theta + nk;
    for (int64_t i = 0; i < m; ++i) {
        const double h = a->h_obs + (double)i * step;
        const double eta = std::exp(log_eta_param(sp, theta, h));
        // psi = eta (2 + eta): d psi / d log eta = eta (2 + 2 eta)
        const double g_log = gpsi[i] * eta * (2.0 + 2.0 * eta);
        KnotPos kp = knot_pos(sp, h);
        g_theta[kp.j] += g_log * (1.0 - kp.f);
        g_theta[kp.j + 1] += g_log * kp.f;
        for (int32_t l = 0; l < nl; ++l) {
            const double over = layer_overlap(sp, l, h);
            if (over > 0.0) g_theta[nk + l] += g_log * over / (H[l] * H[l]);
        }
    }
}

}  // namespace ckv
