/*
 * ckv_oracle.c -- plain FP64 CPU oracle for Cherenkov photon-bunch generation
 * and propagation through a refracting plane-parallel atmosphere to telescope
 * spheres (arXiv 2006.14927, App. A flow; App. B propagation tail; sec. 3.3
 * atmosphere tables; sec. 2 fiducial spheres).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library: it is written
 * separately from the definitions, step by step, in FP64, and is meant to be
 * read against the paper.  Build with -ffp-contract=off (no FMA contraction):
 * bunch counts must come out of the same IEEE operations as on the GPU.
 *
 * Where the paper is silent the following readings are used:
 *  - yield: Frank-Tamm with an index independent of wavelength, expectation
 *    value (no Poisson draw), band [lambda_min, lambda_max];
 *  - one index per step, taken at the step midpoint (yield, threshold, angle);
 *  - beta constant along a step, from total energy and mass;
 *  - n_b = ceil(N / bunch_size) equal sub-steps, photons per bunch = N / n_b;
 *  - emission point uniform inside its sub-step; emission time t0 + s/(beta c);
 *  - azimuth uniform, frame from Duff et al. (JCGT 2017) orthonormal basis;
 *  - wavelength drawn from a 1/lambda^2 spectrum by inverse CDF;
 *  - plane-parallel atmosphere, psi = n^2-1 piecewise linear between nodes of a
 *    uniform grid anchored at the observation level (sec. 3.3.2 fast
 *    interpolation); refraction from cumulative moments of psi (a 5-term
 *    binomial series of the exact Snell integrals);
 *  - drop rules: w <= w_min, emission below the observation level or at/above
 *    the table top; each reason counted;
 *  - sphere test on the infinite line through the ground point along the
 *    observed direction; tangent counts as a hit; several hits allowed.
 *
 * Units: m, ns, MeV, nm.  Directions (u, v, w) with w = -dh/ds (> 0 downward).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C_M_PER_NS 0.299792458
#define OR_ALPHA 7.2973525693e-3          /* CODATA 2018 */
#define OR_MASS_E 0.51099895000           /* MeV, CODATA 2018 */
#define OR_MASS_MU 105.6583755            /* MeV, CODATA 2018 */
#define OR_TWO_PI (2.0 * 3.14159265358979323846)

enum { OR_DROP_MASS = 0, OR_DROP_THRESHOLD, OR_DROP_NONFINITE, OR_DROP_BELOW_OBS,
       OR_DROP_ABOVE_TOP, OR_DROP_UPWARD, OR_DROP_GRAZING, OR_N_DROP };

typedef struct {
    /* atmosphere: uniform grid h_i = h_obs + i*step, i = 0..n_nodes-1 */
    int64_t n_nodes;
    double h_obs, step;
    const double* psi;     /* n_nodes */
    const double* P;       /* 5 x n_nodes: P[(j-1)*n_nodes + i] = int_{h_obs}^{h_i} psi^j dh */
    /* telescopes */
    int32_t n_tel;
    const double *tx, *ty, *tr;
    /* parameters */
    double bunch_size, lambda_min, lambda_max, w_min;
    uint64_t seed;
    int32_t grazing_exact;   /* 1: bunches with 0 < w <= w_min are traced exactly, not dropped */
    const double* h_nodes;   /* NULL: uniform nodes h_obs + i*step; else node altitudes
                                (ascending, h_nodes[0] = h_obs), found by binary search */
    double earth_radius;     /* 0: plane-parallel atmosphere; > 0: spherical shells of this
                                radius (curved variant, every bunch traced exactly) */
} or_config;

typedef struct {
    const double *x0, *y0, *h0, *u, *v, *w, *len, *t0, *energy;
    const uint8_t* ptype;
    const uint32_t* shower_id;  /* RNG counter word 2 */
    const uint32_t* seg_id;     /* RNG counter word 1: index of the step in its shower */
    const int32_t* bucket;      /* output group (shower index) */
    const double* t_ref;        /* per-segment copy of its shower's time origin */
    int64_t n;
} or_segments;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers: */
/* as easy as 1, 2, 3"): 10 rounds of a 4-word Feistel-like network; each      */
/* round multiplies words 0 and 2 by fixed constants, swaps, and xors in the   */
/* key; the key is advanced by two Weyl constants between rounds.             */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0,1): (r + 1/2) / 2^32, exact in FP64 */
static double or_uniform(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------- */
/* Atmosphere tables (sec. 3.3.1 linear interpolation of tabulated quantities; */
/* sec. 3.3.2 fine tables with uniform altitude steps built once at start).    */
/* ------------------------------------------------------------------------- */

/* number of uniform nodes h_obs + i*step that lie inside [alt[0], alt[n-1]] */
int64_t or_grid_size(const double* alt, int64_t n, double h_obs, double step)
{
    if (n < 2 || !(step > 0.0) || h_obs < alt[0] || h_obs >= alt[n - 1]) return -1;
    int64_t m = (int64_t)floor((alt[n - 1] - h_obs) / step) + 1;
    while (m > 1 && h_obs + (double)(m - 1) * step > alt[n - 1]) --m;
    return m;
}

/* eta at altitude h by linear interpolation in the input table; a node of the
   input is returned exactly (sec. 3.3.1: search the bracketing pair, then
   interpolate linearly) */
static double or_eta_at(const double* alt, const double* eta, int64_t n, double h)
{
    int64_t lo = 0, hi = n - 1;
    while (hi - lo > 1) {               /* binary search: alt[lo] <= h < alt[hi] */
        int64_t mid = (lo + hi) / 2;
        if (alt[mid] <= h) lo = mid; else hi = mid;
    }
    if (h == alt[lo]) return eta[lo];
    if (h == alt[hi]) return eta[hi];
    double f = (h - alt[lo]) / (alt[hi] - alt[lo]);
    return eta[lo] + f * (eta[hi] - eta[lo]);
}

/* psi_i = n_i^2 - 1 = eta_i (2 + eta_i) on the uniform grid, and the cumulative
   moments P_j(h_i) = int_{h_obs}^{h_i} psi(h)^j dh, j = 1..5, for psi linear
   inside each cell: the cell integral of (a + (b-a) t)^j is
   step/(j+1) * sum_{m=0..j} a^(j-m) b^m.  Summed upward from h_obs. */
int or_build_tables(const double* alt, const double* eta, int64_t n, double h_obs,
                    double step, int64_t n_nodes, double* psi, double* P)
{
    for (int64_t i = 0; i < n_nodes; ++i) {
        double h = h_obs + (double)i * step;
        double e = or_eta_at(alt, eta, n, h);
        psi[i] = e * (2.0 + e);
    }
    for (int j = 1; j <= 5; ++j) P[(j - 1) * n_nodes + 0] = 0.0;
    for (int64_t i = 0; i + 1 < n_nodes; ++i) {
        double a = psi[i], b = psi[i + 1];
        for (int j = 1; j <= 5; ++j) {
            double sum = 0.0;
            for (int m = 0; m <= j; ++m) sum += pow(a, j - m) * pow(b, m);
            P[(j - 1) * n_nodes + i + 1] = P[(j - 1) * n_nodes + i] + step / (j + 1) * sum;
        }
    }
    return 0;
}

/* psi(h) and P_1..P_5(h): locate the cell directly from the uniform step (no
   search), interpolate psi linearly, and add the partial-cell integral. */
/* altitude of node i, the table top, and the cell holding h (clamped into the
   table): c with h_c <= h < h_{c+1}, fraction f = (h - h_c)/(h_{c+1} - h_c) and
   dz = f * (h_{c+1} - h_c).  Uniform tables: x = (h - h_obs) / step, c = floor(x),
   f = x - c (sec. 3.3.2, no search); node tables: binary search for the
   bracketing pair (sec. 3.3.1, as RPOL does), then the same linear fraction. */
static double or_node_h(const or_config* cf, int64_t i)
{
    return cf->h_nodes ? cf->h_nodes[i] : cf->h_obs + (double)i * cf->step;
}

static double or_h_top(const or_config* cf) { return or_node_h(cf, cf->n_nodes - 1); }

static void or_cell(const or_config* cf, double h, int64_t* c_out, double* f_out, double* dz_out)
{
    int64_t N = cf->n_nodes;
    double h_top = or_h_top(cf);
    double hc = h < cf->h_obs ? cf->h_obs : (h > h_top ? h_top : h);
    if (!cf->h_nodes) {
        double x = (hc - cf->h_obs) * (1.0 / cf->step);
        int64_t i = (int64_t)floor(x);
        if (i > N - 2) i = N - 2;
        *c_out = i;
        *f_out = x - (double)i;
        *dz_out = *f_out * cf->step;
        return;
    }
    int64_t lo = 0, hi = N - 1;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (cf->h_nodes[mid] <= hc) lo = mid; else hi = mid;
    }
    double width = cf->h_nodes[lo + 1] - cf->h_nodes[lo];
    *c_out = lo;
    *dz_out = hc - cf->h_nodes[lo];
    *f_out = *dz_out / width;
}

void or_lookup(const or_config* cf, double h, double* psi_out, double P_out[5])
{
    int64_t N = cf->n_nodes;
    int64_t i;
    double f, dz;
    or_cell(cf, h, &i, &f, &dz);
    double a = cf->psi[i], b = cf->psi[i + 1];
    double p = a + f * (b - a);
    *psi_out = p;
    if (P_out) {
        for (int j = 1; j <= 5; ++j) {
            double sum = 0.0;
            for (int m = 0; m <= j; ++m) sum += pow(a, j - m) * pow(p, m);
            P_out[j - 1] = cf->P[(j - 1) * N + i] + dz / (j + 1) * sum;
        }
    }
}

/* Vertical depth (atmospheric thickness, g/cm^2) on the same uniform grid: the
   tabulated thickness interpolated linearly in altitude, as the index is
   (sec. 3.3.1: one search per altitude serves density, thickness and index;
   sec. 3.3.2: fine uniform tables built once). */
int or_build_depth(const double* alt, const double* depth, int64_t n, double h_obs, double step,
                   int64_t n_nodes, double* T)
{
    for (int64_t i = 0; i < n_nodes; ++i)
        T[i] = or_eta_at(alt, depth, n, h_obs + (double)i * step);
    return 0;
}

/* Tables on the input's own nodes (the standard interpolation of sec. 3.3.1,
   without resampling): the observation level, then every input altitude above
   it.  psi and the cumulative moments as for the uniform grid, with the width
   of each cell.  Returns the node count, or -1 (obs level outside the table). */
int64_t or_build_node_tables(const double* alt, const double* eta, int64_t n, double h_obs,
                             double* h_nodes, double* psi, double* P, int64_t cap)
{
    if (n < 2 || h_obs < alt[0] || h_obs >= alt[n - 1]) return -1;
    int64_t m = 0;
    h_nodes[m++] = h_obs;
    for (int64_t i = 0; i < n; ++i)
        if (alt[i] > h_obs && m < cap) h_nodes[m++] = alt[i];
    for (int64_t i = 0; i < m; ++i) {
        double e = or_eta_at(alt, eta, n, h_nodes[i]);
        psi[i] = e * (2.0 + e);
    }
    for (int j = 1; j <= 5; ++j) P[(j - 1) * m + 0] = 0.0;
    for (int64_t i = 0; i + 1 < m; ++i) {
        double a = psi[i], b = psi[i + 1], width = h_nodes[i + 1] - h_nodes[i];
        for (int j = 1; j <= 5; ++j) {
            double sum = 0.0;
            for (int q = 0; q <= j; ++q) sum += pow(a, j - q) * pow(b, q);
            P[(j - 1) * m + i + 1] = P[(j - 1) * m + i] + width / (j + 1) * sum;
        }
    }
    return m;
}

/* ------------------------------------------------------------------------- */
/* Per-step setup (App. A: for each step the number of emitted photons is     */
/* computed; the step is cut into sub-steps with one bunch of about 5 photons */
/* each).                                                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t status;       /* -1 emits: >= 0 drop reason */
    int64_t n_b;
    double N, photons, cos_t, sin_t, beta, ds, inv_beta_c, n_mid, psi_mid;
    double D[3], b1[3], b2[3];   /* physical direction (u, v, -w) and its frame */
} or_setup;

/* Curved variant: x, y horizontal at the array origin, z along the origin's
   vertical from sea level, the Earth's centre at (0, 0, -R).  The altitude of
   a point is its distance from the centre minus R, written without the
   cancellation of sqrt(...) - R. */
double or_curved_altitude(double R, double x, double y, double z)
{
    double q = x * x + y * y;
    double rz = R + z;
    double r = sqrt(q + rz * rz);
    return (q + z * (2.0 * R + z)) / (r + R);
}

double or_frank_tamm_k(double lambda_min_nm, double lambda_max_nm)
{
    /* 2 pi alpha (1/l1 - 1/l2), in photons per metre for sin^2(theta) = 1 */
    return OR_TWO_PI * OR_ALPHA * (1.0 / lambda_min_nm - 1.0 / lambda_max_nm) * 1e9;
}

void or_segment_setup(const or_config* cf, const or_segments* sg, int64_t i, or_setup* st)
{
    memset(st, 0, sizeof(*st));
    st->status = -1;
    double E = sg->energy[i], L = sg->len[i];
    double vals[9] = {sg->x0[i], sg->y0[i], sg->h0[i], sg->u[i], sg->v[i], sg->w[i], L,
                      sg->t0[i], E};
    for (int q = 0; q < 9; ++q)
        if (!isfinite(vals[q])) { st->status = OR_DROP_NONFINITE; return; }
    if (!(L > 0.0)) { st->status = OR_DROP_NONFINITE; return; }
    double m = sg->ptype[i] == 1 ? OR_MASS_MU : OR_MASS_E;
    double r = m / E;
    double r2 = r * r;                       /* 1/gamma^2 = 1 - beta^2 */
    if (!(r2 < 1.0)) { st->status = OR_DROP_MASS; return; }
    double h_mid;
    if (cf->earth_radius > 0.0) {
        /* curved: the altitude of the step's midpoint above the spherical shells */
        double hl = 0.5 * L;
        h_mid = or_curved_altitude(cf->earth_radius, sg->x0[i] + hl * sg->u[i],
                                   sg->y0[i] + hl * sg->v[i], sg->h0[i] - hl * sg->w[i]);
    } else {
        h_mid = sg->h0[i] - (0.5 * L) * sg->w[i];
    }
    double psi;
    or_lookup(cf, h_mid, &psi, NULL);
    double n2 = 1.0 + psi;
    double num = psi - n2 * r2;              /* = (1 - r2) n^2 - 1 = beta^2 n^2 - 1 */
    if (!(num > 0.0)) { st->status = OR_DROP_THRESHOLD; return; }
    double sin2 = num / (n2 * (1.0 - r2));   /* 1 - 1/(beta n)^2 */
    double K = or_frank_tamm_k(cf->lambda_min, cf->lambda_max);
    double N = (K * L) * sin2;
    double nb = ceil(N / cf->bunch_size);
    st->n_b = (int64_t)nb;
    st->N = N;
    st->photons = N / nb;
    st->psi_mid = psi;
    st->n_mid = sqrt(n2);
    st->cos_t = 1.0 / sqrt((1.0 - r2) * n2);
    st->sin_t = sqrt(sin2);
    st->beta = sqrt(1.0 - r2);
    st->ds = L / nb;
    st->inv_beta_c = 1.0 / (st->beta * OR_C_M_PER_NS);
    /* frame around D (Duff et al. 2017, branchless orthonormal basis) */
    double Dx = sg->u[i], Dy = sg->v[i], Dz = -sg->w[i];
    double sgn = copysign(1.0, Dz);
    double a = -1.0 / (sgn + Dz);
    double b = Dx * Dy * a;
    st->D[0] = Dx; st->D[1] = Dy; st->D[2] = Dz;
    st->b1[0] = 1.0 + sgn * Dx * Dx * a; st->b1[1] = sgn * b; st->b1[2] = -sgn * Dx;
    st->b2[0] = b; st->b2[1] = sgn + Dy * Dy * a; st->b2[2] = -Dy;
}

/* ------------------------------------------------------------------------- */
/* Propagation to the observation level (App. B: emission direction replaced */
/* by the observed one through n sin(theta) conservation, ground position     */
/* displaced by the refraction offset, travel time added to emission time).   */
/* Exact Snell integrals for a stratified medium, expanded in                 */
/* x = (psi - psi_e) / (n_e^2 w^2):                                           */
/*   horizontal advance = (tan theta_e) sum_k a_k q^k D_k,                    */
/*   c * time = 1/(n_e w) sum_k a_k q^k (n_e^2 D_k + D_{k+1}),                */
/* with D_k = int_{h_obs}^{h_e} (psi - psi_e)^k dh and a_k the coefficients  */
/* of (1+x)^(-1/2).                                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    double x_g, y_g, T, u_o, v_o, w_o, n_e, psi_e, S;
} or_prop;

void or_propagate(const or_config* cf, double x_e, double y_e, double h_e, double u, double v,
                  double w, or_prop* pr)
{
    static const double a_k[5] = {1.0, -1.0 / 2.0, 3.0 / 8.0, -5.0 / 16.0, 35.0 / 128.0};
    static const double binom[6][6] = {{1}, {1, 1}, {1, 2, 1}, {1, 3, 3, 1}, {1, 4, 6, 4, 1},
                                        {1, 5, 10, 10, 5, 1}};
    double psi_e, P[5];
    or_lookup(cf, h_e, &psi_e, P);
    double dh = h_e - cf->h_obs;
    double Pj[6] = {dh, P[0], P[1], P[2], P[3], P[4]};   /* P_0 = h_e - h_obs */
    double D[6];
    for (int k = 0; k <= 5; ++k) {
        double sum = 0.0;
        for (int j = 0; j <= k; ++j) sum += binom[k][j] * pow(-psi_e, k - j) * Pj[j];
        D[k] = sum;
    }
    double ne2 = 1.0 + psi_e;
    double ne = sqrt(ne2);
    double q = 1.0 / (ne2 * w * w);
    double S = 0.0, Tsum = 0.0;
    for (int k = 0; k <= 4; ++k) {
        double c = a_k[k] * pow(q, k);
        S += c * D[k];
        Tsum += c * (ne2 * D[k] + D[k + 1]);
    }
    double n_obs = sqrt(1.0 + cf->psi[0]);
    pr->S = S;
    pr->x_g = x_e + (u / w) * S;
    pr->y_g = y_e + (v / w) * S;
    pr->T = Tsum / (OR_C_M_PER_NS * ne * w);
    pr->u_o = u * ne / n_obs;
    pr->v_o = v * ne / n_obs;
    pr->w_o = sqrt(1.0 - pr->u_o * pr->u_o - pr->v_o * pr->v_o);
    pr->n_e = ne;
    pr->psi_e = psi_e;
}

/* Exact propagation, cell by cell (the rare-bunch slow path of sec. 4.3.1 and
   App. C, done exactly instead of by the series): with Snell's invariant
   p = n_e sin(theta_e) and psi linear in each cell, s = n cos(theta) satisfies
   s^2 = n_e^2 w^2 + psi - psi_e, linear in altitude, and over a cell of
   height dz between s_t (top) and s_b (bottom)
     horizontal advance   int p / s dh        = 2 p dz / (s_t + s_b),
     c * travel time      int (s^2 + p^2) / s dh
                          = (2/3) dz (s_t^2 + s_t s_b + s_b^2) / (s_t + s_b) + 2 p^2 dz / (s_t + s_b).
   The ray goes down from h_e through the partial cell and then every full cell
   to h_obs; a downward ray never turns (n grows downward). */
void or_propagate_exact(const or_config* cf, double x_e, double y_e, double h_e, double u,
                        double v, double w, or_prop* pr)
{
    int64_t N = cf->n_nodes;
    double psi_e;
    or_lookup(cf, h_e, &psi_e, NULL);
    double ne2 = 1.0 + psi_e, ne = sqrt(ne2);
    double sin_e = sqrt(u * u + v * v);
    double p = ne * sin_e;
    double s0sq = ne2 * w * w;            /* s^2 at emission */
    int64_t c;
    double f_c, dz_c;
    or_cell(cf, h_e, &c, &f_c, &dz_c);
    double X = 0.0, cT = 0.0;
    double h_top = h_e, s_t = sqrt(s0sq);
    for (int64_t i = c; i >= 0; --i) {
        double h_b = or_node_h(cf, i);
        double dz = h_top - h_b;
        double s_b = sqrt(s0sq + (cf->psi[i] - psi_e));
        if (dz > 0.0) {
            double den = s_t + s_b;
            X += 2.0 * p * dz / den;
            cT += (2.0 / 3.0) * dz * (s_t * s_t + s_t * s_b + s_b * s_b) / den + 2.0 * p * p * dz / den;
        }
        h_top = h_b;
        s_t = s_b;
    }
    double n_obs = sqrt(1.0 + cf->psi[0]);
    pr->S = X;
    pr->x_g = sin_e > 0.0 ? x_e + (u / sin_e) * X : x_e;
    pr->y_g = sin_e > 0.0 ? y_e + (v / sin_e) * X : y_e;
    pr->T = cT / OR_C_M_PER_NS;
    pr->u_o = u * ne / n_obs;
    pr->v_o = v * ne / n_obs;
    pr->w_o = sqrt(1.0 - pr->u_o * pr->u_o - pr->v_o * pr->v_o);
    pr->n_e = ne;
    pr->psi_e = psi_e;
}

void or_propagate_exact_many(const or_config* cf, int64_t m, const double* in, double* out)
{
    for (int64_t q = 0; q < m; ++q) {
        const double* pp = in + 6 * q;
        or_prop pr;
        or_propagate_exact(cf, pp[0], pp[1], pp[2], pp[3], pp[4], pp[5], &pr);
        double* o = out + 9 * q;
        o[0] = pr.x_g; o[1] = pr.y_g; o[2] = pr.T; o[3] = pr.u_o; o[4] = pr.v_o;
        o[5] = pr.w_o; o[6] = pr.n_e; o[7] = pr.psi_e; o[8] = pr.S;
    }
}


/* ------------------------------------------------------------------------- */
/* Curved atmosphere (spherical shells of radius R; the large-zenith variant). */
/* The index depends on the altitude h = r - R only (r the distance from the  */
/* Earth's centre C), so a ray stays in the plane of C, its emission point and */
/* its direction, and keeps the Bouguer invariant K = n r sin(zeta), zeta the  */
/* angle from the local vertical.  With s = sqrt(n^2 r^2 - K^2) the polar      */
/* angle swept about C and the optical path down to the observation sphere    */
/* r_obs = R + h_obs are                                                      */
/*   theta = int K / (r s) dr,     c T = int n^2 r / s dr.                    */
/* s^2 is taken relative to the emission point, s^2 = s_e^2 + M(h) - M(h_e)   */
/* with M = n^2 r^2, M(h) - M(h_e) = (h - h_e)(r + r_e) + psi r^2 - psi_e r_e^2 */
/* and s_e = n_e (r_e cos zeta_e), which keeps it accurate for grazing rays.   */
/* psi is linear in h inside each table cell; over a cell, s^2 is nearly      */
/* linear in h, so the substitution h = h_b + dh (u^2 - s_b^2)/(s_t^2 - s_b^2) */
/* (u from s_b to s_t) removes the 1/s behaviour:                             */
/*   int F / s dh = 2 dh / (s_t^2 - s_b^2) int F(h(u)) u / s(h(u)) du,        */
/* evaluated with 8-point Gauss-Legendre in u.  While n r grows with r (air   */
/* at the Earth's radius: no ducting) the ray reaches the ground iff s^2 > 0  */
/* there, and a ray with cos zeta_e <= 0 moves outward for good.              */
/* The array is treated as planar: the ground point's x, y and the arrival    */
/* direction's x, y components enter the same sphere test as the flat path.   */
/* Returns -1, OR_DROP_UPWARD or OR_DROP_GRAZING (the ray turns above ground). */
/* ------------------------------------------------------------------------- */
static const double or_gl8_x[4] = {0.18343464249564980493947614236018,
                                   0.52553240991632898581773904918925,
                                   0.79666647741362673959155393647583,
                                   0.96028985649753623168356086856947};
static const double or_gl8_w[4] = {0.36268378337836198296515044927720,
                                   0.31370664587788728733796220198660,
                                   0.22238103445337447054435599442624,
                                   0.10122853629037625915253135430996};

int or_propagate_curved(const or_config* cf, double x_e, double y_e, double z_e, double u,
                        double v, double w, or_prop* pr)
{
    double R = cf->earth_radius;
    double rz = R + z_e;
    double r_e = sqrt(x_e * x_e + y_e * y_e + rz * rz);
    double h_e = or_curved_altitude(R, x_e, y_e, z_e);
    /* r_e cos(zeta_e) with zeta_e measured from the downward local vertical */
    double mu_num = w * rz - u * x_e - v * y_e;
    memset(pr, 0, sizeof(*pr));
    if (!(mu_num > 0.0)) return OR_DROP_UPWARD;
    double psi_e;
    or_lookup(cf, h_e, &psi_e, NULL);
    double ne2 = 1.0 + psi_e, ne = sqrt(ne2);
    /* r_e sin(zeta_e) = |(P_e - C) x D|, D = (u, v, -w) */
    double Lx = -y_e * w - rz * v, Ly = rz * u + x_e * w, Lz = x_e * v - y_e * u;
    double K = ne * sqrt(Lx * Lx + Ly * Ly + Lz * Lz);
    double s2e = ne2 * (mu_num * mu_num);
    double Mr_e = psi_e * r_e * r_e;
    double r_obs = R + cf->h_obs;
    double s2g = s2e + ((cf->h_obs - h_e) * (r_obs + r_e) + cf->psi[0] * r_obs * r_obs - Mr_e);
    if (!(s2g > 0.0)) return OR_DROP_GRAZING;
    int64_t c;
    double f_c, dz_c;
    or_cell(cf, h_e, &c, &f_c, &dz_c);
    double theta = 0.0, opt = 0.0;
    double h_t = h_e, psi_t = psi_e, s2t = s2e, s_t = sqrt(s2e);
    for (int64_t i = c; i >= 0; --i) {
        double h_b = or_node_h(cf, i);
        double psi_b = cf->psi[i];
        double r_b = R + h_b;
        double s2b = i == 0 ? s2g : s2e + ((h_b - h_e) * (r_b + r_e) + psi_b * r_b * r_b - Mr_e);
        double s_b = sqrt(s2b);
        double dh = h_t - h_b;
        if (dh > 0.0 && s2t != s2b) {   /* (a cell of zero s^2 span adds ~dh/s: nothing) */
            double g = (psi_t - psi_b) / dh;
            double mid = 0.5 * (s_t + s_b), half = 0.5 * (s_t - s_b);
            double a_th = 0.0, a_op = 0.0;
            for (int q = 0; q < 8; ++q) {
                double xq = q < 4 ? -or_gl8_x[3 - q] : or_gl8_x[q - 4];
                double wq = q < 4 ? or_gl8_w[3 - q] : or_gl8_w[q - 4];
                double uq = mid + half * xq;
                double hq = h_b + dh * ((uq * uq - s2b) / (s2t - s2b));
                double psq = psi_b + g * (hq - h_b);
                double rq = R + hq;
                double s2q = s2e + ((hq - h_e) * (rq + r_e) + psq * rq * rq - Mr_e);
                double ratio = uq / sqrt(s2q);
                a_th += wq * (K / rq) * ratio;
                a_op += wq * ((1.0 + psq) * rq) * ratio;
            }
            theta += dh / (s_t + s_b) * a_th;
            opt += dh / (s_t + s_b) * a_op;
        }
        h_t = h_b;
        psi_t = psi_b;
        s2t = s2b;
        s_t = s_b;
    }
    /* ground point: rotate the emission point's radial direction by theta
       towards the ray's tangential direction, at radius r_obs */
    double rho[3] = {x_e / r_e, y_e / r_e, rz / r_e};
    double mu = mu_num / r_e;
    double tp[3] = {u + mu * rho[0], v + mu * rho[1], -w + mu * rho[2]};
    double sz = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
    for (int a = 0; a < 3; ++a) tp[a] = sz > 0.0 ? tp[a] / sz : 0.0;
    double ct = cos(theta), sn = sin(theta);
    double rg[3], tg[3];
    for (int a = 0; a < 3; ++a) {
        rg[a] = ct * rho[a] + sn * tp[a];
        tg[a] = -sn * rho[a] + ct * tp[a];
    }
    double n_obs = sqrt(1.0 + cf->psi[0]);
    double sin_g = K / (n_obs * r_obs), cos_g = sqrt(s2g) / (n_obs * r_obs);
    pr->x_g = r_obs * rg[0];
    pr->y_g = r_obs * rg[1];
    pr->u_o = -cos_g * rg[0] + sin_g * tg[0];
    pr->v_o = -cos_g * rg[1] + sin_g * tg[1];
    pr->w_o = sqrt(1.0 - pr->u_o * pr->u_o - pr->v_o * pr->v_o);
    pr->T = opt / OR_C_M_PER_NS;
    pr->n_e = ne;
    pr->psi_e = psi_e;
    pr->S = r_obs * theta;
    return -1;
}

/* rows of 10: status, then the 9 fields of or_propagate_many */
void or_propagate_curved_many(const or_config* cf, int64_t m, const double* in, double* out)
{
    for (int64_t q = 0; q < m; ++q) {
        const double* pp = in + 6 * q;
        or_prop pr;
        int st = or_propagate_curved(cf, pp[0], pp[1], pp[2], pp[3], pp[4], pp[5], &pr);
        double* o = out + 10 * q;
        o[0] = st;
        o[1] = pr.x_g; o[2] = pr.y_g; o[3] = pr.T; o[4] = pr.u_o; o[5] = pr.v_o;
        o[6] = pr.w_o; o[7] = pr.n_e; o[8] = pr.psi_e; o[9] = pr.S;
    }
}

/* ------------------------------------------------------------------------- */
/* One bunch k of a step: sub-step emission point, direction on the Cherenkov */
/* cone, wavelength, drop rules, propagation.                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t status;      /* -1 propagated; >= 0 drop reason */
    uint32_t r[4];
    double x_e, y_e, h_e, t_e, u, v, w, lambda, photons;
    or_prop pr;
    double t;            /* arrival time minus the shower's t_ref */
} or_bunch;

void or_make_bunch(const or_config* cf, const or_segments* sg, int64_t i, const or_setup* st,
                   int64_t k, or_bunch* bn)
{
    memset(bn, 0, sizeof(*bn));
    uint32_t ctr[4] = {(uint32_t)k, sg->seg_id[i], sg->shower_id[i], 0u};
    uint32_t key[2] = {(uint32_t)cf->seed, (uint32_t)(cf->seed >> 32)};
    or_philox4x32_10(ctr, key, bn->r);
    double u0 = or_uniform(bn->r[0]), u1 = or_uniform(bn->r[1]), u2 = or_uniform(bn->r[2]);
    /* emission point: uniform inside sub-step k */
    double s = ((double)k + u0) * st->ds;
    bn->x_e = sg->x0[i] + s * sg->u[i];
    bn->y_e = sg->y0[i] + s * sg->v[i];
    bn->h_e = sg->h0[i] - s * sg->w[i];
    bn->t_e = sg->t0[i] + s * st->inv_beta_c;
    /* direction: cone of half-angle theta_c around D, azimuth phi */
    double phi = OR_TWO_PI * u1;
    double cp = cos(phi), sp = sin(phi);
    double C[3];
    for (int a = 0; a < 3; ++a)
        C[a] = st->cos_t * st->D[a] + st->sin_t * (cp * st->b1[a] + sp * st->b2[a]);
    bn->u = C[0]; bn->v = C[1]; bn->w = -C[2];
    /* wavelength from dN/dlambda ~ 1/lambda^2 on [l1, l2] */
    double il1 = 1.0 / cf->lambda_min, il2 = 1.0 / cf->lambda_max;
    bn->lambda = 1.0 / (il1 - u2 * (il1 - il2));
    bn->photons = st->photons;
    double h_top = or_h_top(cf);
    if (cf->earth_radius > 0.0) {
        /* curved: drops on the true altitude; every bunch traced exactly */
        double z_e = bn->h_e;
        bn->h_e = or_curved_altitude(cf->earth_radius, bn->x_e, bn->y_e, z_e);
        if (bn->h_e < cf->h_obs) { bn->status = OR_DROP_BELOW_OBS; return; }
        if (bn->h_e >= h_top) { bn->status = OR_DROP_ABOVE_TOP; return; }
        bn->status = or_propagate_curved(cf, bn->x_e, bn->y_e, z_e, bn->u, bn->v, bn->w, &bn->pr);
        if (bn->status < 0) bn->t = bn->t_e + bn->pr.T - sg->t_ref[i];
        return;
    }
    if (bn->h_e < cf->h_obs) { bn->status = OR_DROP_BELOW_OBS; return; }
    if (bn->h_e >= h_top) { bn->status = OR_DROP_ABOVE_TOP; return; }
    if (bn->w <= 0.0) { bn->status = OR_DROP_UPWARD; return; }
    int grazing = bn->w <= cf->w_min;
    if (grazing && !cf->grazing_exact) { bn->status = OR_DROP_GRAZING; return; }
    bn->status = -1;
    if (grazing)
        or_propagate_exact(cf, bn->x_e, bn->y_e, bn->h_e, bn->u, bn->v, bn->w, &bn->pr);
    else
        or_propagate(cf, bn->x_e, bn->y_e, bn->h_e, bn->u, bn->v, bn->w, &bn->pr);
    bn->t = bn->t_e + bn->pr.T - sg->t_ref[i];
}

/* sphere test: line through (x_g, y_g, h_obs) along the observed direction;
   it meets the sphere of radius R centred at (X, Y, h_obs) iff the squared
   distance of closest approach dx^2+dy^2-b^2 is <= R^2 */
double or_sphere_disc(double x_g, double y_g, double u_o, double v_o, double X, double Y,
                      double R)
{
    double dx = x_g - X, dy = y_g - Y;
    double b = dx * u_o + dy * v_o;
    return b * b - (dx * dx + dy * dy - R * R);
}

/* ------------------------------------------------------------------------- */
/* Whole run: every step, every bunch, every telescope (brute force).         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t seg;        /* index into the segment arrays of the call */
    int64_t k;          /* bunch index inside its step */
    int32_t tel, bucket;
    double rec[8];      /* dx, dy, u_o, v_o, t, h_e, photons, lambda */
    double disc;
} or_hit;

typedef struct {
    or_hit* hits;
    int64_t n_hits, cap;
    int64_t n_bunches;
    int64_t n_emitting;
    int64_t drops[OR_N_DROP];
} or_result;

static void or_push(or_result* r, const or_hit* h)
{
    if (r->n_hits == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 1024;
        r->hits = (or_hit*)realloc(r->hits, (size_t)r->cap * sizeof(or_hit));
    }
    r->hits[r->n_hits++] = *h;
}

static void or_run_range(const or_config* cf, const or_segments* sg, int64_t lo, int64_t hi,
                         or_result* r, int64_t* n_b_out)
{
    for (int64_t i = lo; i < hi; ++i) {
        or_setup st;
        or_segment_setup(cf, sg, i, &st);
        if (n_b_out) n_b_out[i] = st.status >= 0 ? 0 : st.n_b;
        if (st.status >= 0) { r->drops[st.status]++; continue; }
        r->n_emitting++;
        r->n_bunches += st.n_b;
        for (int64_t k = 0; k < st.n_b; ++k) {
            or_bunch bn;
            or_make_bunch(cf, sg, i, &st, k, &bn);
            if (bn.status >= 0) { r->drops[bn.status]++; continue; }
            for (int32_t t = 0; t < cf->n_tel; ++t) {
                double disc = or_sphere_disc(bn.pr.x_g, bn.pr.y_g, bn.pr.u_o, bn.pr.v_o,
                                             cf->tx[t], cf->ty[t], cf->tr[t]);
                if (disc >= 0.0) {
                    or_hit h;
                    h.seg = i; h.k = k; h.tel = t; h.bucket = sg->bucket[i];
                    h.rec[0] = bn.pr.x_g - cf->tx[t];
                    h.rec[1] = bn.pr.y_g - cf->ty[t];
                    h.rec[2] = bn.pr.u_o;
                    h.rec[3] = bn.pr.v_o;
                    h.rec[4] = bn.t;
                    h.rec[5] = bn.h_e;
                    h.rec[6] = bn.photons;
                    h.rec[7] = bn.lambda;
                    h.disc = disc;
                    or_push(r, &h);
                }
            }
        }
    }
}

/* Runs all segments; hits are returned in segment order, bunch order, then
   telescope order.  Grouping by (bucket, telescope) is left to the caller.
   Threads split the segments into contiguous ranges; results are joined in
   range order, so the output does not depend on the thread count. */
/* ------------------------------------------------------------------------- */
/* Longitudinal profile of Cherenkov photon production (the CERLDE output,     */
/* sec. 4.3.3 and 5.2.2): for every shower, the photons and bunches emitted in  */
/* bins of vertical depth X of the emission point, bin b = floor(X / width)    */
/* (multiplied by 1/width), counting every bunch emitted inside the tables,    */
/* h_obs <= h_e < h_top, whatever its direction.  X(h_e) is read from the depth */
/* table exactly as psi is: x = (h - h_obs) / step, i = floor(x), linear in f.  */
/* ------------------------------------------------------------------------- */
static void or_profile_range(const or_config* cf, const or_segments* sg, const double* T,
                             double inv_width, int32_t n_bins, int64_t lo, int64_t hi,
                             double* photons, int64_t* bunches)
{
    int64_t N = cf->n_nodes;
    double h_top = or_h_top(cf);
    uint32_t key[2] = {(uint32_t)cf->seed, (uint32_t)(cf->seed >> 32)};
    for (int64_t i = lo; i < hi; ++i) {
        or_setup st;
        or_segment_setup(cf, sg, i, &st);
        if (st.status >= 0) continue;
        for (int64_t k = 0; k < st.n_b; ++k) {
            uint32_t ctr[4] = {(uint32_t)k, sg->seg_id[i], sg->shower_id[i], 0u}, r[4];
            or_philox4x32_10(ctr, key, r);
            double s = ((double)k + or_uniform(r[0])) * st.ds;
            double h_e = sg->h0[i] - s * sg->w[i];
            if (h_e < cf->h_obs || h_e >= h_top) continue;
            int64_t c;
            double f, dz;
            or_cell(cf, h_e, &c, &f, &dz);
            double X = T[c] + f * (T[c + 1] - T[c]);
            int64_t b = (int64_t)floor(X * inv_width);
            if (b < 0) b = 0;
            if (b > n_bins - 1) b = n_bins - 1;
            int64_t g = (int64_t)sg->bucket[i] * n_bins + b;
            photons[g] += st.photons;
            bunches[g] += 1;
        }
    }
}

/* photons and bunches: n_groups x n_bins each, zeroed here */
int or_profile(const or_config* cf, const or_segments* sg, const double* T, double width,
               int32_t n_bins, int32_t n_groups, int nthreads, double* photons, int64_t* bunches)
{
    if (nthreads < 1) nthreads = 1;
    size_t m = (size_t)n_groups * n_bins;
    double* ph = (double*)calloc((size_t)nthreads * m, sizeof(double));
    int64_t* bu = (int64_t*)calloc((size_t)nthreads * m, sizeof(int64_t));
    double inv_width = 1.0 / width;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = sg->n * t / nthreads, hi = sg->n * (t + 1) / nthreads;
        or_profile_range(cf, sg, T, inv_width, n_bins, lo, hi, ph + (size_t)t * m, bu + (size_t)t * m);
    }
    for (size_t q = 0; q < m; ++q) {
        double a = 0.0;
        int64_t c = 0;
        for (int t = 0; t < nthreads; ++t) { a += ph[(size_t)t * m + q]; c += bu[(size_t)t * m + q]; }
        photons[q] = a;
        bunches[q] = c;
    }
    free(ph);
    free(bu);
    return 0;
}

or_result* or_run(const or_config* cf, const or_segments* sg, int nthreads, int64_t* n_b_out)
{
    or_result* res = (or_result*)calloc(1, sizeof(or_result));
    if (nthreads < 1) nthreads = 1;
    or_result* parts = (or_result*)calloc((size_t)nthreads, sizeof(or_result));
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = sg->n * t / nthreads, hi = sg->n * (t + 1) / nthreads;
        or_run_range(cf, sg, lo, hi, &parts[t], n_b_out);
    }
    for (int t = 0; t < nthreads; ++t) {
        for (int64_t h = 0; h < parts[t].n_hits; ++h) or_push(res, &parts[t].hits[h]);
        res->n_bunches += parts[t].n_bunches;
        res->n_emitting += parts[t].n_emitting;
        for (int d = 0; d < OR_N_DROP; ++d) res->drops[d] += parts[t].drops[d];
        free(parts[t].hits);
    }
    free(parts);
    return res;
}

int64_t or_result_n_hits(const or_result* r) { return r->n_hits; }
void or_result_counters(const or_result* r, int64_t* out /* 2 + OR_N_DROP */)
{
    out[0] = r->n_bunches;
    out[1] = r->n_emitting;
    for (int d = 0; d < OR_N_DROP; ++d) out[2 + d] = r->drops[d];
}
void or_result_copy(const or_result* r, int64_t* seg, int64_t* k, int32_t* tel, int32_t* bucket,
                    double* rec /* n x 8 */, double* disc)
{
    for (int64_t h = 0; h < r->n_hits; ++h) {
        seg[h] = r->hits[h].seg; k[h] = r->hits[h].k;
        tel[h] = r->hits[h].tel; bucket[h] = r->hits[h].bucket;
        memcpy(rec + 8 * h, r->hits[h].rec, 8 * sizeof(double));
        disc[h] = r->hits[h].disc;
    }
}
void or_result_free(or_result* r)
{
    if (!r) return;
    free(r->hits);
    free(r);
}

/* Details of selected bunches, rows of 28 doubles:
   status, n_b, photons, cos_t, sin_t, x_e, y_e, h_e, t_e, u, v, w, lambda,
   x_g, y_g, T, u_o, v_o, w_o, t, n_e, psi_e, S, r0, r1, r2, r3, ds */
void or_bunch_details(const or_config* cf, const or_segments* sg, int64_t m,
                      const int64_t* seg, const int64_t* k, double* out /* m x 28 */)
{
    for (int64_t q = 0; q < m; ++q) {
        double* o = out + 28 * q;
        or_setup st;
        or_segment_setup(cf, sg, seg[q], &st);
        for (int z = 0; z < 28; ++z) o[z] = NAN;
        o[0] = st.status; o[1] = (double)st.n_b; o[2] = st.photons;
        o[3] = st.cos_t; o[4] = st.sin_t;
        if (st.status >= 0 || k[q] < 0 || k[q] >= st.n_b) continue;
        or_bunch bn;
        or_make_bunch(cf, sg, seg[q], &st, k[q], &bn);
        o[0] = bn.status;
        o[5] = bn.x_e; o[6] = bn.y_e; o[7] = bn.h_e; o[8] = bn.t_e;
        o[9] = bn.u; o[10] = bn.v; o[11] = bn.w; o[12] = bn.lambda;
        if (bn.status < 0) {
            o[13] = bn.pr.x_g; o[14] = bn.pr.y_g; o[15] = bn.pr.T;
            o[16] = bn.pr.u_o; o[17] = bn.pr.v_o; o[18] = bn.pr.w_o; o[19] = bn.t;
            o[20] = bn.pr.n_e; o[21] = bn.pr.psi_e; o[22] = bn.pr.S;
        }
        for (int a = 0; a < 4; ++a) o[23 + a] = (double)bn.r[a];
        o[27] = st.ds;
    }
}

/* per-segment setup table: rows of 16 doubles
   status, n_b, N, photons, cos_t, sin_t, beta, ds, inv_beta_c, n_mid, b1[3], b2[3] */
void or_segment_details(const or_config* cf, const or_segments* sg, double* out)
{
    for (int64_t i = 0; i < sg->n; ++i) {
        or_setup st;
        or_segment_setup(cf, sg, i, &st);
        double* o = out + 16 * i;
        o[0] = st.status; o[1] = (double)st.n_b; o[2] = st.N; o[3] = st.photons;
        o[4] = st.cos_t; o[5] = st.sin_t; o[6] = st.beta; o[7] = st.ds; o[8] = st.inv_beta_c;
        o[9] = st.n_mid;
        for (int a = 0; a < 3; ++a) { o[10 + a] = st.b1[a]; o[13 + a] = st.b2[a]; }
    }
}

/* lookups at many altitudes: out rows psi, P1..P5 */
void or_lookup_many(const or_config* cf, int64_t m, const double* h, double* out)
{
    for (int64_t q = 0; q < m; ++q) {
        double P[5];
        or_lookup(cf, h[q], out + 6 * q, P);
        for (int j = 0; j < 5; ++j) out[6 * q + 1 + j] = P[j];
    }
}

/* propagate arbitrary photons: rows of 9 = x_g, y_g, T, u_o, v_o, w_o, n_e, psi_e, S */
void or_propagate_many(const or_config* cf, int64_t m, const double* in /* m x 6 */, double* out)
{
    for (int64_t q = 0; q < m; ++q) {
        const double* p = in + 6 * q;
        or_prop pr;
        or_propagate(cf, p[0], p[1], p[2], p[3], p[4], p[5], &pr);
        double* o = out + 9 * q;
        o[0] = pr.x_g; o[1] = pr.y_g; o[2] = pr.T; o[3] = pr.u_o; o[4] = pr.v_o;
        o[5] = pr.w_o; o[6] = pr.n_e; o[7] = pr.psi_e; o[8] = pr.S;
    }
}

/* ------------------------------------------------------------------------- */
/* Soft telescope response (differentiation pattern; no counterpart in the    */
/* paper).  For shower s and telescope k:                                     */
/*   S_sk = sum over bunches of photons * Phi(z),                             */
/*   A_sk = sum over bunches of photons * Phi(z) * t,                         */
/*   z = (R_k^2 - rho^2) / (2 R_k sigma),  rho^2 = dx^2 + dy^2 - b^2,         */
/* rho the distance of closest approach of the observed ray to the centre and */
/* Phi the standard normal CDF.  Bunch counts are frozen (n_b_frozen per      */
/* step): yield, angle and photons per bunch follow the current tables, the   */
/* sub-step positions do not.  A step whose current sin^2(theta_c) <= 0       */
/* emits nothing.  Every telescope is visited (brute force).                  */
/* ------------------------------------------------------------------------- */
static double or_phi(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

void or_soft(const or_config* cf, const or_segments* sg, const int64_t* n_b_frozen, double sigma,
             int32_t n_showers, int nthreads, double* S, double* A)
{
    int64_t nsk = (int64_t)n_showers * cf->n_tel;
    if (nthreads < 1) nthreads = 1;
    double* part = (double*)calloc((size_t)nthreads * 2 * nsk, sizeof(double));
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
    for (int th = 0; th < nthreads; ++th) {
        double* pS = part + (size_t)th * 2 * nsk;
        double* pA = pS + nsk;
        int64_t lo = sg->n * th / nthreads, hi = sg->n * (th + 1) / nthreads;
        for (int64_t i = lo; i < hi; ++i) {
            if (n_b_frozen[i] <= 0) continue;
            or_setup st;
            or_segment_setup(cf, sg, i, &st);
            if (st.status >= 0) continue;          /* no light at the current tables */
            /* frozen count: photons per bunch and sub-step length use n_b_frozen */
            double nb = (double)n_b_frozen[i];
            st.n_b = n_b_frozen[i];
            st.photons = st.N / nb;
            st.ds = sg->len[i] / nb;
            for (int64_t k = 0; k < st.n_b; ++k) {
                or_bunch bn;
                or_make_bunch(cf, sg, i, &st, k, &bn);
                if (bn.status >= 0) continue;
                for (int32_t t = 0; t < cf->n_tel; ++t) {
                    double dx = bn.pr.x_g - cf->tx[t], dy = bn.pr.y_g - cf->ty[t];
                    double b = dx * bn.pr.u_o + dy * bn.pr.v_o;
                    double rho2 = dx * dx + dy * dy - b * b;
                    double R = cf->tr[t];
                    double z = (R * R - rho2) / (2.0 * R * sigma);
                    double W = or_phi(z);
                    if (W == 0.0) continue;
                    int64_t q = (int64_t)sg->bucket[i] * cf->n_tel + t;
                    pS[q] += bn.photons * W;
                    pA[q] += bn.photons * W * bn.t;
                }
            }
        }
    }
    for (int64_t q = 0; q < nsk; ++q) {
        double s = 0.0, a = 0.0;
        for (int th = 0; th < nthreads; ++th) {
            s += part[(size_t)th * 2 * nsk + q];
            a += part[(size_t)th * 2 * nsk + nsk + q];
        }
        S[q] = s;
        A[q] = a;
    }
    free(part);
}

/* Parameterised atmosphere: log eta(h) = log eta0 - sum_l overlap([0,h], layer l)/H_l
   + Lambda(h), with Lambda the linear interpolant of knot values at
   h_j = j * knot_top / (n_knots - 1), constant above knot_top.  The last
   layer extends upward.  theta = (knots[n_knots], H[n_layers]). */
double or_log_eta_param(double eta0, int32_t n_layers, const double* bounds, int32_t n_knots,
                        double knot_top, const double* theta, double h)
{
    const double* knots = theta;
    const double* H = theta + n_knots;
    double depth = 0.0;
    for (int32_t l = 0; l < n_layers; ++l) {
        double top = (l + 1 < n_layers) ? bounds[l + 1] : INFINITY;
        double hi = h < top ? h : top;
        double over = hi - bounds[l];
        if (over > 0.0) depth += over / H[l];
    }
    double hc = h < knot_top ? h : knot_top;
    double dk = knot_top / (double)(n_knots - 1);
    double x = hc / dk;
    int32_t j = (int32_t)floor(x);
    if (j > n_knots - 2) j = n_knots - 2;
    if (j < 0) j = 0;
    double f = x - (double)j;
    double lam = knots[j] + f * (knots[j + 1] - knots[j]);
    return log(eta0) - depth + lam;
}

void or_eta_param_many(double eta0, int32_t n_layers, const double* bounds, int32_t n_knots,
                       double knot_top, const double* theta, int64_t m, const double* h, double* eta)
{
    for (int64_t q = 0; q < m; ++q)
        eta[q] = exp(or_log_eta_param(eta0, n_layers, bounds, n_knots, knot_top, theta, h[q]));
}
