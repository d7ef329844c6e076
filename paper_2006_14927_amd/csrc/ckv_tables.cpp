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
    return CKV_OK;
}

int build_array_grid(ckv_array* arr)
{
    const int32_t n = arr->n_tel;
    double rmax = 0, xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int32_t k = 0; k < n; ++k) {
        double reach = arr->r[k] / kGridWLo;
        rmax = std::max(rmax, arr->r[k]);
        xmin = std::min(xmin, arr->x[k] - reach);
        xmax = std::max(xmax, arr->x[k] + reach);
        ymin = std::min(ymin, arr->y[k] - reach);
        ymax = std::max(ymax, arr->y[k] + reach);
    }
    double extent = std::max(xmax - xmin, ymax - ymin);
    double margin = 0.01 + 1e-9 * extent;
    double cell = std::max(2.0 * rmax, extent / 1024.0);
    xmin -= margin; ymin -= margin;
    int32_t nx = (int32_t)std::ceil((xmax + margin - xmin) / cell) + 1;
    int32_t ny = (int32_t)std::ceil((ymax + margin - ymin) / cell) + 1;
    arr->gx0 = xmin;
    arr->gy0 = ymin;
    arr->cell = cell;
    arr->inv_cell = 1.0 / cell;
    arr->nx = nx;
    arr->ny = ny;
    arr->cell_off.assign((size_t)nx * ny + 1, 0);
    std::vector<std::vector<uint16_t>> lists((size_t)nx * ny);
    for (int32_t k = 0; k < n; ++k) {
        double reach = arr->r[k] / kGridWLo + margin;
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
                    lists[(size_t)ix * ny + iy].push_back((uint16_t)k);
            }
    }
    arr->cell_list.clear();
    for (size_t c = 0; c < lists.size(); ++c) {
        arr->cell_off[c] = (int32_t)arr->cell_list.size();
        arr->cell_list.insert(arr->cell_list.end(), lists[c].begin(), lists[c].end());
    }
    arr->cell_off[lists.size()] = (int32_t)arr->cell_list.size();
    if (arr->cell_list.empty()) arr->cell_list.push_back(0);
    return CKV_OK;
}

}  // namespace ckv
