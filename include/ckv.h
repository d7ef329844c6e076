/*
 * ckv.h -- C ABI of the MI355X Cherenkov photon-bunch library.
 *
 * What it computes (arXiv 2006.14927): for every charged-particle track step
 * the number of Cherenkov photons is computed and split into bunches of about
 * five photons, one bunch per sub-step (App. A); every bunch is bent by
 * atmospheric refraction and propagated to the observation level, where its
 * position, observed direction and arrival time are obtained (App. B); the
 * bunches that cross a telescope's fiducial sphere are written out per
 * telescope (sec. 2; App. A, TELOUT).  Atmospheric quantities come from fine
 * tables with a uniform altitude step, built once (sec. 3.3.2 "fast
 * interpolation"), from a user-supplied profile (sec. 2, external profiles).
 *
 * Conventions: units m, ns, MeV, nm.  x, y horizontal, h altitude.  Directions
 * are (u, v, w) = (dx/ds, dy/ds, -dh/ds): w > 0 is downward.  The atmosphere
 * is plane-parallel, or (params->earth_radius_m > 0) made of spherical shells
 * around the Earth's centre (0, 0, -R): then h is the Cartesian height along
 * the array origin's vertical and the altitude of a point is its distance from
 * the centre minus R.
 *
 * Errors: every call returns CKV_OK (0) or a negative code; no exception
 * crosses the ABI.  ckv_last_error() gives a message for the calling thread.
 * Arguments are validated on the host before anything is enqueued.  Conditions
 * only visible on the device (capacity overflow, dropped bunches, bad segment
 * values) do not fail the call: they are reported in ckv_result.
 *
 * Ownership: the caller owns every large device buffer (segments, records,
 * offsets, result, workspace, soft bunch list).  Handles (ckv_atmo, ckv_array) are immutable
 * after creation, own only their small host and device tables, and may be
 * shared by concurrent runs on different streams.  ckv_run is re-entrant
 * given distinct workspaces and outputs.
 */
#ifndef CKV_H
#define CKV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CKV_VERSION 114

enum {
    CKV_OK = 0,
    CKV_ERR_ARG = -1,       /* invalid argument (null pointer, negative size, bad value) */
    CKV_ERR_TABLE = -2,     /* invalid atmosphere profile or telescope list */
    CKV_ERR_CAPACITY = -3,  /* workspace smaller than ckv_workspace_size() */
    CKV_ERR_HIP = -4,       /* HIP runtime error (launch, copy, allocation of handle tables) */
    CKV_ERR_NOMEM = -5      /* host allocation failed */
};

/* arithmetic of the per-bunch path (the per-step bunch count is always FP64) */
enum { CKV_FP64 = 0, CKV_MIXED = 1 };

/* particle types: mass used for beta */
enum { CKV_ELECTRON = 0, CKV_MUON = 1 };

/* reasons counted in ckv_result.drops */
enum {
    CKV_DROP_MASS = 0,       /* step: total energy <= mass */
    CKV_DROP_THRESHOLD = 1,  /* step: beta n <= 1 at the step midpoint (no light) */
    CKV_DROP_NONFINITE = 2,  /* step: non-finite value or length <= 0 */
    CKV_DROP_BELOW_OBS = 3,  /* bunch: emitted below the observation level */
    CKV_DROP_ABOVE_TOP = 4,  /* bunch: emitted at or above the table top */
    CKV_DROP_UPWARD = 5,     /* bunch: w <= 0, never reaches the ground */
    CKV_DROP_GRAZING = 6,    /* bunch: 0 < w <= w_min */
    CKV_N_DROP = 8
};

typedef struct ckv_atmo ckv_atmo;
typedef struct ckv_array ckv_array;

/* Message of the last failing call on this thread ("" if none). */
const char* ckv_last_error(void);
/* CKV_VERSION of the loaded library. */
int ckv_version(void);

/* ---------------------------------------------------------------------------
 * Atmosphere (sec. 3.3.1 tabulated refractive index vs altitude, linear
 * interpolation between tabulated points; sec. 3.3.2 fine tables with a
 * uniform step built once; sec. 2 external profiles).
 *
 * alt_m[n] strictly increasing, eta[n] = n-1 >= 0, host memory, copied.
 * The library samples eta by linear interpolation onto the uniform grid
 * h_i = obs_level_m + i*step_m inside [alt_m[0], alt_m[n-1]] (a grid node that
 * coincides with an input node takes its value exactly), with step_m = 0
 * meaning alt_m[1]-alt_m[0].  It stores psi = n^2-1 at the nodes and the
 * cumulative moments P_j(h_i) = integral from obs level to h_i of psi^j dh,
 * j = 1..5, for psi linear inside each cell; these drive the refraction
 * offset and travel time.  Tables are uploaded to the current HIP device.
 * Errors: CKV_ERR_ARG (null, n < 2, step < 0), CKV_ERR_TABLE (altitudes not
 * increasing, eta < 0 or non-finite, obs level outside the table, fewer
 * than 2 nodes), CKV_ERR_HIP.
 * ------------------------------------------------------------------------- */
int ckv_atmo_create(const double* alt_m, const double* eta, int64_t n, double obs_level_m,
                    double step_m, ckv_atmo** out);
/* As ckv_atmo_create, with the vertical depth (atmospheric thickness, g/cm^2)
   tabulated at the same altitudes: depth_gcm2[n], finite, non-increasing with
   altitude, host memory, copied.  The library samples it onto the same uniform
   grid the same way as eta (sec. 3.3.1: one search per altitude serves the
   thickness and the index; sec. 3.3.2: fine uniform tables built once), which
   enables the longitudinal profile of ckv_run (depth_bin_gcm2 > 0).
   Errors: as ckv_atmo_create; CKV_ERR_TABLE also for a depth that increases
   with altitude or is not finite. */
int ckv_atmo_create_with_depth(const double* alt_m, const double* eta, const double* depth_gcm2,
                               int64_t n, double obs_level_m, double step_m, ckv_atmo** out);
/* Host copy of the depth at the grid nodes, depth[n_nodes].  CKV_ERR_ARG if
   the handle has no depth table. */
int ckv_atmo_depth(const ckv_atmo* atmo, double* depth);
/* Bins of width bin_gcm2 that cover depths [0, X(h_obs)]: floor(X(h_obs) /
   bin_gcm2) + 1 (X(h_obs) times 1/bin_gcm2).  CKV_ERR_ARG without a depth
   table, for bin_gcm2 <= 0, or above CKV_MAX_PROFILE_BINS bins. */
#define CKV_MAX_PROFILE_BINS 128
int ckv_profile_bins(const ckv_atmo* atmo, double bin_gcm2, int32_t* n_bins);
/* Node tables: the same tables on the profile's own altitudes (the observation
   level, then every alt_m[i] above it), looked up by a binary search for the
   bracketing pair and linear interpolation (sec. 3.3.1, the standard RPOL
   interpolation), instead of resampling onto a uniform grid (sec. 3.3.2).
   2 <= n <= CKV_MAX_NODE_TABLE.  For the table-lookup ablation: ckv_run takes
   such a handle with tile_segments 0 or 32 and neither the profile nor the
   exact grazing path; ckv_atmo_info reports step 0.  Errors: as
   ckv_atmo_create. */
#define CKV_MAX_NODE_TABLE 4096
int ckv_atmo_create_nodes(const double* alt_m, const double* eta, int64_t n, double obs_level_m,
                          ckv_atmo** out);
/* Node altitudes of the handle, h_nodes[n_nodes] (uniform grids too). */
int ckv_atmo_nodes(const ckv_atmo* atmo, double* h_nodes);
/* Grid of the handle: node count, observation level, step. */
int ckv_atmo_info(const ckv_atmo* atmo, int64_t* n_nodes, double* obs_level_m, double* step_m);
/* Host copies of the tables: psi[n_nodes], P[5*n_nodes] with
   P[(j-1)*n_nodes + i] = P_j(h_i).  Either pointer may be NULL. */
int ckv_atmo_tables(const ckv_atmo* atmo, double* psi, double* P);
int ckv_atmo_destroy(ckv_atmo* atmo);

/* ---------------------------------------------------------------------------
 * Telescopes (sec. 2: fiducial spheres at positions on the ground).
 * Centres (x_m, y_m) at the observation level, sphere radii r_m > 0; host
 * memory, copied.  1 <= n_tel <= CKV_MAX_TEL.  The library builds a uniform
 * 2-D candidate grid so each bunch tests only nearby spheres.
 * Errors: CKV_ERR_ARG, CKV_ERR_TABLE (non-finite or r <= 0), CKV_ERR_HIP.
 * ------------------------------------------------------------------------- */
#define CKV_MAX_TEL 1024
int ckv_array_create(const double* x_m, const double* y_m, const double* r_m, int32_t n_tel,
                     ckv_array** out);
int ckv_array_destroy(ckv_array* arr);

/* ---------------------------------------------------------------------------
 * Run inputs.  All pointers below are DEVICE pointers.
 * ------------------------------------------------------------------------- */

/* Track steps, structure of arrays, n entries each, grouped by shower
   (App. A: each particle track is subdivided into steps).  Start point
   (x0, y0, h0) [m], unit direction (u, v, w) with w = -dh/ds, length [m],
   start time t0 [ns], total energy [MeV], particle type (CKV_ELECTRON or
   CKV_MUON; charge 1).  step_id (optional, NULL to leave out): the random-
   number counter word of each step (below: it replaces seg_id_base[s] + j), so
   the steps of a shower may be stored in any order -- e.g. sorted by altitude
   for table locality (sec. 6, cache behaviour) -- and every bunch keeps its
   random numbers; records then still name steps by their index in these
   arrays. */
typedef struct {
    const double *x0, *y0, *h0, *u, *v, *w, *length, *t0, *energy;
    const uint8_t* ptype;
    int64_t n;
    const uint32_t* step_id;
} ckv_segments;

/* Showers: steps of shower s are [seg_offsets[s], seg_offsets[s+1]),
   seg_offsets[0] = 0, seg_offsets[n_showers] = n.  t_ref[s] is subtracted
   from arrival times.  Random numbers of bunch k of the step with index j in
   its shower come from Philox4x32-10 with counter
   (k, seg_id_base[s] + j, shower_ids[s], 0), or (k, step_id[i], shower_ids[s],
   0) for the step at index i when segments->step_id is given, and the 64-bit
   seed as key
   (sec. 5.2: runs reproduce the same random sequence); shower_ids NULL means
   shower_ids[s] = s, seg_id_base NULL means 0.  Splitting a shower's steps
   into several runs with the matching seg_id_base gives the same bunches. */
typedef struct {
    const int64_t* seg_offsets;   /* n_showers + 1 */
    const double* t_ref;          /* n_showers */
    const uint32_t* shower_ids;   /* n_showers or NULL */
    const int64_t* seg_id_base;   /* n_showers or NULL */
    int32_t n_showers;
} ckv_showers;

typedef struct {
    double bunch_size;     /* photons per bunch target (App. A: typically 5), > 0 */
    double lambda_min_nm;  /* Cherenkov band, 0 < lambda_min < lambda_max */
    double lambda_max_nm;
    double w_min;          /* bunches with w <= w_min are dropped (0 <= w_min < 1) */
    uint64_t seed;         /* Philox key */
    int32_t precision;     /* CKV_FP64 or CKV_MIXED */
    int32_t tile_segments; /* steps per emit tile: 8, 16, 32 or 64; 0 = default (32) */
    int32_t grid;          /* bunch-kernel workgroups, 0 = one per compute unit */
    int32_t waves_per_group; /* bunch-kernel waves per workgroup: 1, 2, 4, 8 or 16 (FP64:
                              <= 8); 0 = the most that fit the LDS; a value that does not
                              fit is lowered to one that does */
    void* event_begin;     /* optional hipEvent_t recorded on the stream just before */
    void* event_end;       /* and just after the bunch kernel (profiling); NULL = none */
    double depth_bin_gcm2; /* > 0: also accumulate the longitudinal photon-production
                              profile in bins of this width (needs an atmosphere with a
                              depth table); 0 = no profile */
    int32_t grazing_exact; /* 0: bunches with 0 < w <= w_min are dropped (counted);
                              1: they are propagated exactly, cell by cell in FP64 through
                              the index table, instead of by the moment series (the slow
                              path for rare bunches, sec. 4.3.1 and App. C) */
    int32_t reserved;      /* must be 0 */
    double earth_radius_m; /* 0: plane-parallel atmosphere.  > 0: curved variant for large
                              zenith angles: spherical shells of this radius (Earth: 6.371e6);
                              step midpoints and emission points take their true altitude,
                              and every bunch is traced exactly (Bouguer's invariant
                              n r sin(zeta), cell by cell through the index table, FP64)
                              down to the observation sphere h = h_obs, where the ground
                              point's x, y and the arrival direction's x, y components enter
                              the sphere test (the array is taken as planar).  Drops: below
                              the observation level or above the table on the true altitude;
                              upward = moving away from the centre; grazing = the ray turns
                              above the observation sphere.  Needs uniform tables,
                              tile_segments 0 or 32, no profile, grazing_exact 0; not for the
                              soft response. */
} ckv_params;

/* Device-side report, written by ckv_run (the caller syncs the stream before
   reading it). */
typedef struct {
    int64_t n_bunches;       /* bunches generated: sum of n_b over the run's steps */
    int64_t n_hits;          /* sphere crossings of the run's steps: the capacity that
                                holds them all (written or not) */
    int64_t n_records;       /* records written (all n_hits unless overflow) */
    int64_t n_emitting;      /* steps with at least one bunch */
    int64_t n_tiles;         /* emit tiles processed */
    int64_t drops[CKV_N_DROP];
    int64_t resume_step;     /* overflow: first step (index in the segment arrays) whose
                                records were not written; n otherwise */
    int32_t resume_shower;   /* overflow: the shower of resume_step; n_showers otherwise */
    int32_t overflow;        /* 1: the crossings did not fit the capacity: the records
                                of the steps before resume_step are written, complete and
                                in canonical order, and tel_offsets describe them; the
                                steps from resume_step on were computed (they are in the
                                counters) but not written: resume there (ckv_cursor).
                                The prefix is the longest that fits while the crossings
                                fit the workspace's staging (capacity plus 64 per bunch-
                                kernel wave); beyond that tiles finishing out of order
                                may end it earlier, possibly at the first step */
    int32_t error;           /* bit 0: seg_offsets not non-decreasing or out of range,
                                or a resume cursor outside the steps; bit 1: a tile of
                                tile_segments steps held >= 2^30 bunches (its bunches
                                were skipped) */
    int32_t reserved;
} ckv_result;

/* Where a run starts (App. A, TELOUT: the bunches that hit are written as the
   steps are processed; a run cut short by a full output continues where it
   stopped): the steps before `step` (an index in the segment arrays) are left
   out, `shower` is the shower holding it.  Bunches keep their random numbers
   (the counter uses the step's index in its shower), so the records of a run
   resumed at the cursor its predecessor reported, appended per (shower,
   telescope) to the predecessor's, are the records of one uninterrupted run. */
typedef struct {
    int64_t step;
    int32_t shower;
    int32_t reserved;        /* 0 */
} ckv_cursor;

/* Output.  records: capacity x 8 floats per record
     (x - X_tel, y - Y_tel, u_obs, v_obs, t - t_ref, h_emit, photons, lambda)
   [m, m, -, -, ns, m, photons, nm].  Records of shower s and telescope k are
   records[tel_offsets[s*n_tel + k] .. tel_offsets[s*n_tel + k + 1]), in
   ascending (step, bunch) order.  ids (optional, NULL to skip): capacity x 2
   int64 per record = (index of the step in the segment arrays, bunch k).
   Longitudinal profile (the CERLDE output, sec. 4.3.3 and 5.2.2; only when
   params->depth_bin_gcm2 > 0): n_showers x n_bins each (ckv_profile_bins),
   photons and bunches emitted per shower in bins of vertical depth X of the
   emission point, bin floor(X * (1/width)), counting every bunch emitted at
   h_obs <= h < h_top whatever its direction; X is the depth table read like
   the index, in FP64 without contraction, so bins match the FP64 definition
   exactly.  Overwritten by each run (photon sums in FP64 by atomics: their
   rounding order varies). */
typedef struct {
    float* records;
    int64_t* ids;
    int64_t capacity;
    int64_t* tel_offsets;    /* n_showers * n_tel + 1 */
    ckv_result* result;
    double* profile_photons;   /* n_showers * n_bins, or NULL without a profile */
    int64_t* profile_bunches;  /* n_showers * n_bins, or NULL without a profile */
} ckv_output;

/* Bytes of device workspace ckv_run needs for these sizes. */
size_t ckv_workspace_size(int64_t n_segments, int32_t n_showers, int32_t n_tel,
                          int64_t capacity, const ckv_params* params);

/* Generate and propagate every bunch of every step, test it against every
   telescope sphere, and write the crossing records per (shower, telescope).
   Fully asynchronous on `stream` (a hipStream_t; NULL = default stream);
   enqueues kernels only, so it can be captured into a HIP graph.
   workspace: device memory of ws_bytes >= ckv_workspace_size(...), any
   content.  resume_from (host memory, may be NULL = from the first step):
   start at that cursor, typically the resume_step/resume_shower an overflowing
   run reported.  When the crossings exceed the capacity the run writes a
   complete prefix of its steps and reports where to resume (ckv_result).
   Errors (synchronous): CKV_ERR_ARG for null pointers, n < 0, n_showers < 1,
   bad params, a cursor with step outside [0, n] or shower outside
   [0, n_showers), a profile asked for without a depth table, with too many
   bins or without its output arrays; CKV_ERR_CAPACITY for a small workspace;
   CKV_ERR_HIP if a launch fails. */
int ckv_run(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
            const ckv_atmo* atmo, const ckv_array* arr, void* workspace, size_t ws_bytes,
            ckv_output* out, const ckv_cursor* resume_from, void* stream);

/* ckv_run without a workspace argument, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc).  The workspace is a static device array of
   CKV_NOALLOC_SCRATCH_MIB MiB inside the library: each GPU the library runs on
   holds its own copy until the process ends, and this call allocates nothing
   (no hipMalloc, hipFree or allocating library routine).  The caller still
   passes the inputs and the output buffers.  Every call on one GPU shares that
   GPU's array, which keeps the last call's contents (each run starts by
   resetting what it reads, as ckv_run does with any workspace): calls that
   overlap on one GPU -- concurrent streams or threads -- race and give wrong
   results; serialise them.  Results are identical to ckv_run's with the same
   arguments.  Errors: as ckv_run; CKV_ERR_CAPACITY when the run needs more than
   the array holds (ckv_noalloc_workspace_size() > CKV_NOALLOC_SCRATCH_MIB MiB;
   then use ckv_run). */
#define CKV_NOALLOC_SCRATCH_MIB 256
int ckv_run_noalloc(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                    const ckv_atmo* atmo, const ckv_array* arr, ckv_output* out,
                    const ckv_cursor* resume_from, void* stream);
/* Bytes of the static array ckv_run_noalloc would use for these sizes on the
   current device (0 for invalid sizes). */
size_t ckv_noalloc_workspace_size(int64_t n_segments, int32_t n_showers, int32_t n_tel,
                                  int64_t capacity, const ckv_params* params);

/* Bunch count per step only (the first stage of ckv_run): n_b[i] for every
   step (0 for dropped steps), FP64, the same values ckv_run uses.  n_b is a
   device int64 array of n entries.  Asynchronous on `stream`. */
int ckv_count(const ckv_segments* segs, const ckv_params* params, const ckv_atmo* atmo,
              int64_t* n_b, void* stream);

/* ---------------------------------------------------------------------------
 * Differentiation.  A smooth per-telescope response and its gradient with
 * respect to the atmosphere, for fitting atmospheric profiles to telescope
 * data (no counterpart in the paper; built on the same bunch path).
 *
 * Soft response of shower s at telescope k (sphere centre X, radius R):
 *   S_sk = sum over bunches of photons * Phi(z),
 *   A_sk = sum over bunches of photons * Phi(z) * t,
 *   z = (R^2 - rho^2) / (2 R sigma),
 * rho the distance of closest approach between the observed ray and the
 * sphere centre, Phi the standard normal CDF; Phi(z) = 0 for z < -40 (exactly
 * zero in FP64).  Bunch counts are frozen: n_b_frozen[i] (from ckv_count at a
 * reference atmosphere) fixes the sub-steps, while yield, angle and photons
 * per bunch follow the current atmosphere; a step below threshold at the
 * current atmosphere emits nothing.  S, A and the gradient are computed in FP64
 * (with a bunch list, a mixed-precision pass only selects the bunches).
 * ------------------------------------------------------------------------- */

/* log eta(h) = log eta0 - sum_l overlap([0, h], layer l) / H_l + Lambda(h):
   H_l constant inside layer l = [bounds[l], bounds[l+1]) (the last layer extends
   upward), Lambda the linear interpolant of n_knots values at
   h_j = j * knot_top / (n_knots - 1), constant above knot_top.  The profile is
   sampled at obs_level + i*step up to top.  theta = (knot values, H_l [m]). */
typedef struct {
    double eta0;
    int32_t n_layers;
    int32_t n_knots;
    const double* layer_bounds_m;   /* host, n_layers + 1, increasing */
    double knot_top_m;
    double obs_level_m;
    double step_m;
    double top_m;
} ckv_atmo_param_spec;

/* Atmosphere handle of the parameterised profile at theta (host memory). */
int ckv_atmo_from_params(const ckv_atmo_param_spec* spec, const double* theta, ckv_atmo** out);
/* Chain rule from table gradients to parameters: given dL/dpsi_i (n_nodes) and
   dL/dP_j(h_i) (5 x n_nodes, as from ckv_soft_backward, copied to host) of the
   handle built from (spec, theta), writes dL/dtheta (n_knots + n_layers).
   Host only, synchronous. */
int ckv_atmo_params_backward(const ckv_atmo_param_spec* spec, const double* theta,
                             const ckv_atmo* atmo, const double* g_psi, const double* g_P,
                             double* g_theta);
/* Telescope handle that also carries the candidate grid of the soft response
   for edge width sigma_m > 0 (see ckv_array_create for the other arguments). */
int ckv_array_create_soft(const double* x_m, const double* y_m, const double* r_m, int32_t n_tel,
                          double sigma_m, ckv_array** out);
/* Bunch list of the soft response.  With a list, ckv_soft_forward first screens
   every bunch with the mixed-precision path against spheres of the cut radius
   sqrt(R^2 + 2 R sigma 40) plus 1 cm (far above that path's errors), lists the
   candidates and recomputes only those in FP64 for S and A.  Steps whose light
   provably lands too far from every sphere centre (a bound on the ground ring of
   the step's cone, refraction included) are not screened.  The list thus holds
   every bunch with z >= -40 at some sphere (the ones that enter S, A and the
   gradient) and a few just outside.  Ids are (global step index << 24) | bunch
   index k, in no particular order.  ckv_soft_backward then recomputes only the
   listed bunches (the others contribute exactly zero).  The caller owns both
   device buffers.  *count is the number of candidates (ids beyond capacity are
   not written); the list is complete iff 0 <= *count <= capacity (a bunch index
   of 2^24 or more, or a step index of 2^40 or more, makes it incomplete).  With
   an incomplete list the forward computes S and A from every bunch in FP64 and
   the backward recomputes every bunch. */
typedef struct {
    uint64_t* ids;        /* device, capacity entries */
    int64_t capacity;     /* >= 0 */
    int64_t* count;       /* device, one int64, written by the forward */
} ckv_soft_list;

/* S and A (device, n_showers x n_tel FP64, overwritten).  Same inputs as
   ckv_run plus n_b_frozen (device int64, one per step); the workspace is the
   one ckv_workspace_size(n, n_showers, n_tel, 0, params) gives.  arr must come
   from ckv_array_create_soft.  params->precision is ignored (FP64).  list
   (may be NULL) receives the bunches with a nonzero weight.
   result (device, may be NULL): device-side conditions, in the error word as for
   ckv_run -- bit 0: seg_offsets not non-decreasing or out of range (nothing is
   computed: S = A = 0); bit 1: a 32-step tile whose frozen counts total 2^30
   bunches or more (its bunches are left out); the other fields are zeroed.
   Negative frozen counts emit nothing.  Asynchronous on `stream`. */
int ckv_soft_forward(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                     const ckv_atmo* atmo, const ckv_array* arr, const int64_t* n_b_frozen,
                     double* S, double* A, const ckv_soft_list* list, ckv_result* result,
                     void* workspace, size_t ws_bytes, void* stream);
/* Reverse pass: given dL/dS and dL/dA (device, n_showers x n_tel), recomputes
   bunches from their random numbers and writes dL/dpsi_i (device, n_nodes)
   and dL/dP_j(h_i) (device, 5 x n_nodes), both overwritten; psi_0 also
   carries the observation-level index.  list NULL: every bunch is recomputed.
   list from the ckv_soft_forward of the same inputs: only the listed bunches
   are, when the list is complete (checked on the device; else every bunch);
   a list from other inputs gives a wrong gradient, and ids that name no bunch
   of these inputs are skipped.  result (device, may be NULL): as for
   ckv_soft_forward (bit 0: nothing computed, gradients 0).  Asynchronous on
   `stream`. */
int ckv_soft_backward(const ckv_segments* segs, const ckv_showers* showers, const ckv_params* params,
                      const ckv_atmo* atmo, const ckv_array* arr, const int64_t* n_b_frozen,
                      const double* dL_dS, const double* dL_dA, double* g_psi, double* g_P,
                      const ckv_soft_list* list, ckv_result* result, void* workspace,
                      size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CKV_H */
