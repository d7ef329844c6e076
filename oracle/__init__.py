"""FP64 CPU oracle (test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  It shares no code with the HIP library
(`paper_2006_14927_amd`): the arithmetic lives in `ckv_oracle.c`, written
separately from the paper's description (App. A generation flow, App. B
propagation tail, sec. 3.3 atmosphere tables, sec. 2 telescope spheres), and
this module only marshals arguments and groups hits per (shower, telescope).

Parity pins: every function here is pinned by `tests/test_oracle_*.py`
against closed forms, brute-force tracing, library routines or invariants.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libckv_oracle.so")
_SRC = os.path.join(_HERE, "ckv_oracle.c")

DROP_NAMES = ("mass", "threshold", "nonfinite", "below_obs", "above_top", "upward", "grazing")
W_MIN = 0.1


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


class _Config(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("h_obs", C.c_double), ("step", C.c_double),
                ("psi", C.c_void_p), ("P", C.c_void_p),
                ("n_tel", C.c_int32), ("tx", C.c_void_p), ("ty", C.c_void_p), ("tr", C.c_void_p),
                ("bunch_size", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("w_min", C.c_double), ("seed", C.c_uint64),
                ("grazing_exact", C.c_int32), ("h_nodes", C.c_void_p),
                ("earth_radius", C.c_double)]


class _Segments(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x0", "y0", "h0", "u", "v", "w", "len", "t0",
                                          "energy", "ptype", "shower_id", "seg_id", "bucket",
                                          "t_ref")] + [("n", C.c_int64)]


def _declare(L):
    P, I64, D = C.c_void_p, C.c_int64, C.c_double
    L.or_grid_size.restype = I64
    L.or_grid_size.argtypes = [P, I64, D, D]
    L.or_build_tables.argtypes = [P, P, I64, D, D, I64, P, P]
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_run.restype = P
    L.or_run.argtypes = [C.POINTER(_Config), C.POINTER(_Segments), C.c_int, P]
    L.or_result_n_hits.restype = I64
    L.or_result_n_hits.argtypes = [P]
    L.or_result_counters.argtypes = [P, P]
    L.or_result_copy.argtypes = [P, P, P, P, P, P, P]
    L.or_result_free.argtypes = [P]
    L.or_bunch_details.argtypes = [C.POINTER(_Config), C.POINTER(_Segments), I64, P, P, P]
    L.or_segment_details.argtypes = [C.POINTER(_Config), C.POINTER(_Segments), P]
    L.or_lookup_many.argtypes = [C.POINTER(_Config), I64, P, P]
    L.or_propagate_many.argtypes = [C.POINTER(_Config), I64, P, P]
    L.or_propagate_exact_many.argtypes = [C.POINTER(_Config), I64, P, P]
    L.or_propagate_curved_many.argtypes = [C.POINTER(_Config), I64, P, P]
    L.or_curved_altitude.restype = D
    L.or_curved_altitude.argtypes = [D, D, D, D]
    L.or_sphere_disc.restype = D
    L.or_sphere_disc.argtypes = [D] * 7
    L.or_frank_tamm_k.restype = D
    L.or_frank_tamm_k.argtypes = [D, D]
    L.or_soft.argtypes = [C.POINTER(_Config), C.POINTER(_Segments), P, D, C.c_int32, C.c_int, P, P]
    L.or_eta_param_many.argtypes = [D, C.c_int32, P, C.c_int32, D, P, I64, P, P]
    L.or_build_depth.argtypes = [P, P, I64, D, D, I64, P]
    L.or_build_node_tables.restype = I64
    L.or_build_node_tables.argtypes = [P, P, I64, D, P, P, P, I64]
    L.or_profile.argtypes = [C.POINTER(_Config), C.POINTER(_Segments), P, D, C.c_int32, C.c_int32,
                             C.c_int, P, P]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# atmosphere tables
# ---------------------------------------------------------------------------

@dataclass
class Tables:
    h_obs: float
    step: float
    psi: np.ndarray      # n_nodes
    P: np.ndarray        # (5, n_nodes)
    h_nodes: Optional[np.ndarray] = None   # node altitudes of a non-uniform (search) table

    @property
    def n_nodes(self) -> int:
        return int(self.psi.shape[0])

    @property
    def h_top(self) -> float:
        if self.h_nodes is not None:
            return float(self.h_nodes[-1])
        return self.h_obs + (self.n_nodes - 1) * self.step

    def grid(self) -> np.ndarray:
        if self.h_nodes is not None:
            return self.h_nodes.copy()
        return self.h_obs + np.arange(self.n_nodes) * self.step


def build_depth(alt, depth, t: Tables) -> np.ndarray:
    """Vertical depth [g/cm^2] at the uniform nodes of t (linear in altitude)."""
    alt = np.ascontiguousarray(alt, dtype=np.float64)
    depth = np.ascontiguousarray(depth, dtype=np.float64)
    T = np.empty(t.n_nodes)
    lib().or_build_depth(_p(alt), _p(depth), alt.shape[0], t.h_obs, t.step, t.n_nodes, _p(T))
    return T


def profile_bins(T: np.ndarray, width: float) -> int:
    """Number of depth bins of the given width that cover [0, X(h_obs)]."""
    return int(np.floor(T[0] * (1.0 / width))) + 1


def profile(cfg: "Config", segs, T: np.ndarray, width: float, nthreads: int = 1, seg_id_base=None,
            seg_id=None):
    """Longitudinal photon-production profile: (photons, bunches), each
    (n_showers, n_bins), binned in vertical depth of the emission point."""
    if cfg.earth_radius > 0.0:
        raise ValueError("the profile is defined for the plane-parallel atmosphere")
    sv = SegView(segs, seg_id_base=seg_id_base, seg_id=seg_id)
    T = np.ascontiguousarray(T, dtype=np.float64)
    nb = profile_bins(T, width)
    ph = np.zeros(sv.n_showers * nb)
    bu = np.zeros(sv.n_showers * nb, dtype=np.int64)
    lib().or_profile(C.byref(cfg.c), C.byref(sv.c), _p(T), float(width), nb, sv.n_showers,
                     int(nthreads), _p(ph), _p(bu))
    return ph.reshape(sv.n_showers, nb), bu.reshape(sv.n_showers, nb)


def build_node_tables(alt, eta, h_obs: float) -> Tables:
    """Tables on the input's own altitudes above h_obs (binary-search lookups)."""
    alt = np.ascontiguousarray(alt, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    cap = alt.shape[0] + 1
    hn = np.empty(cap)
    psi = np.empty(cap)
    P = np.empty(5 * cap)
    m = lib().or_build_node_tables(_p(alt), _p(eta), alt.shape[0], h_obs, _p(hn), _p(psi), _p(P), cap)
    if m < 2:
        raise ValueError("observation level outside the atmosphere table")
    P = P[:5 * m].reshape(5, m).copy()
    return Tables(h_obs, float("nan"), psi[:m].copy(), P, hn[:m].copy())


def build_tables(alt, eta, h_obs: float, step: float = 0.0) -> Tables:
    alt = np.ascontiguousarray(alt, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    if step <= 0.0:
        step = float(alt[1] - alt[0])
    n = lib().or_grid_size(_p(alt), alt.shape[0], h_obs, step)
    if n < 2:
        raise ValueError("observation level outside the atmosphere table")
    psi = np.empty(n)
    P = np.empty((5, n))
    lib().or_build_tables(_p(alt), _p(eta), alt.shape[0], h_obs, step, n, _p(psi), _p(P))
    return Tables(h_obs, step, psi, P)


# ---------------------------------------------------------------------------
# configuration and segments
# ---------------------------------------------------------------------------

class Config:
    """Tables + telescopes + parameters, kept alive for the C structure."""

    def __init__(self, tables: Tables, tel_x, tel_y, tel_r, *, bunch_size=5.0,
                 lambda_min=300.0, lambda_max=600.0, seed=0x14927, w_min=W_MIN,
                 grazing_exact=False, earth_radius=0.0):
        self.tables = tables
        self.tx = np.ascontiguousarray(tel_x, dtype=np.float64)
        self.ty = np.ascontiguousarray(tel_y, dtype=np.float64)
        self.tr = np.ascontiguousarray(tel_r, dtype=np.float64)
        self.psi = np.ascontiguousarray(tables.psi)
        self.P = np.ascontiguousarray(tables.P)
        self.h_nodes = None if tables.h_nodes is None else np.ascontiguousarray(tables.h_nodes)
        self.bunch_size, self.lambda_min, self.lambda_max = bunch_size, lambda_min, lambda_max
        self.seed, self.w_min = int(seed), w_min
        self.earth_radius = float(earth_radius)
        self.c = _Config(tables.n_nodes, tables.h_obs, tables.step, _p(self.psi).value,
                         _p(self.P).value, self.tx.shape[0], _p(self.tx).value,
                         _p(self.ty).value, _p(self.tr).value, bunch_size, lambda_min,
                         lambda_max, w_min, self.seed, int(bool(grazing_exact)),
                         None if self.h_nodes is None else _p(self.h_nodes).value,
                         self.earth_radius)

    @property
    def n_tel(self) -> int:
        return int(self.tx.shape[0])

    @staticmethod
    def from_workload(wl, **kw) -> "Config":
        t = build_tables(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
        args = dict(bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                    lambda_max=wl.lambda_max, seed=wl.seed)
        args.update(kw)
        return Config(t, wl.tels.x, wl.tels.y, wl.tels.r, **args)


class SegView:
    """Per-segment arrays in the layout the C oracle reads."""

    def __init__(self, segs, *, seg_id_base: Optional[np.ndarray] = None,
                 seg_id: Optional[np.ndarray] = None):
        n = segs.n
        self.arrs = {}
        for f in segs.FIELDS:
            self.arrs[f] = np.ascontiguousarray(getattr(segs, f), dtype=np.float64)
        self.arrs["ptype"] = np.ascontiguousarray(segs.ptype, dtype=np.uint8)
        offs = np.asarray(segs.seg_offsets, dtype=np.int64)
        counts = np.diff(offs)
        bucket = np.repeat(np.arange(segs.n_showers, dtype=np.int32), counts)
        first = np.repeat(offs[:-1], counts)
        explicit_id = seg_id
        seg_id = (np.arange(n, dtype=np.int64) - first)
        if seg_id_base is not None:
            seg_id = seg_id + np.repeat(np.asarray(seg_id_base, dtype=np.int64), counts)
        if explicit_id is not None:
            seg_id = np.asarray(explicit_id, dtype=np.int64)
        self.arrs["seg_id"] = seg_id.astype(np.uint32)
        self.arrs["shower_id"] = np.repeat(np.asarray(segs.shower_ids, dtype=np.uint32), counts)
        self.arrs["bucket"] = bucket
        self.arrs["t_ref"] = np.repeat(np.asarray(segs.t_ref, dtype=np.float64), counts)
        self.n = n
        self.n_showers = segs.n_showers
        a = self.arrs
        self.c = _Segments(*[_p(a[f]).value for f in segs.FIELDS[:6]],
                           _p(a["length"]).value, _p(a["t0"]).value, _p(a["energy"]).value,
                           _p(a["ptype"]).value, _p(a["shower_id"]).value, _p(a["seg_id"]).value,
                           _p(a["bucket"]).value, _p(a["t_ref"]).value, n)


# ---------------------------------------------------------------------------
# runs
# ---------------------------------------------------------------------------

@dataclass
class Result:
    n_b: np.ndarray          # per segment
    n_bunches: int
    n_emitting: int
    drops: dict
    # hits grouped per (shower, telescope) in ascending (segment, bunch) order
    offsets: np.ndarray      # n_showers * n_tel + 1
    seg: np.ndarray
    k: np.ndarray
    tel: np.ndarray
    bucket: np.ndarray
    rec: np.ndarray          # (n_hits, 8): dx, dy, u_o, v_o, t, h_e, photons, lambda
    disc: np.ndarray


def run(cfg: Config, segs, nthreads: int = 1, seg_id_base=None, seg_id=None) -> Result:
    """All bunches of all steps.  seg_id (optional, per step) overrides the
    step's index in its shower, the RNG counter word 1 (used to run a subset of
    a shower's steps with their original random numbers)."""
    sv = SegView(segs, seg_id_base=seg_id_base, seg_id=seg_id)
    L = lib()
    n_b = np.zeros(sv.n, dtype=np.int64)
    r = L.or_run(C.byref(cfg.c), C.byref(sv.c), int(nthreads), _p(n_b))
    try:
        nh = L.or_result_n_hits(r)
        cnt = np.zeros(2 + len(DROP_NAMES), dtype=np.int64)
        L.or_result_counters(r, _p(cnt))
        seg = np.empty(nh, np.int64)
        k = np.empty(nh, np.int64)
        tel = np.empty(nh, np.int32)
        bucket = np.empty(nh, np.int32)
        rec = np.empty((nh, 8))
        disc = np.empty(nh)
        L.or_result_copy(r, _p(seg), _p(k), _p(tel), _p(bucket), _p(rec), _p(disc))
    finally:
        L.or_result_free(r)
    # group by (shower, telescope); the oracle emits in (segment, bunch, tel)
    # order, so a stable sort on the group key keeps (segment, bunch) order
    key = bucket.astype(np.int64) * cfg.n_tel + tel
    order = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=sv.n_showers * cfg.n_tel)
    offsets = np.zeros(sv.n_showers * cfg.n_tel + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return Result(n_b, int(cnt[0]), int(cnt[1]), dict(zip(DROP_NAMES, map(int, cnt[2:]))),
                  offsets, seg[order], k[order], tel[order], bucket[order], rec[order],
                  disc[order])


BUNCH_FIELDS = ("status", "n_b", "photons", "cos_t", "sin_t", "x_e", "y_e", "h_e", "t_e", "u",
                "v", "w", "lambda", "x_g", "y_g", "T", "u_o", "v_o", "w_o", "t", "n_e", "psi_e",
                "S", "r0", "r1", "r2", "r3", "ds")


def bunch_details(cfg: Config, segs, seg_idx, k, seg_id_base=None) -> dict:
    sv = SegView(segs, seg_id_base=seg_id_base)
    seg_idx = np.ascontiguousarray(seg_idx, dtype=np.int64)
    k = np.ascontiguousarray(k, dtype=np.int64)
    out = np.empty((seg_idx.shape[0], 28))
    lib().or_bunch_details(C.byref(cfg.c), C.byref(sv.c), seg_idx.shape[0], _p(seg_idx), _p(k),
                           _p(out))
    d = {f: out[:, i] for i, f in enumerate(BUNCH_FIELDS)}
    r = np.nan_to_num(out[:, 23:27], nan=0.0)
    d["r"] = r.astype(np.uint64).astype(np.uint32)
    return d


SEG_FIELDS = ("status", "n_b", "N", "photons", "cos_t", "sin_t", "beta", "ds", "inv_beta_c",
              "n_mid", "b1x", "b1y", "b1z", "b2x", "b2y", "b2z")


def segment_details(cfg: Config, segs) -> dict:
    sv = SegView(segs)
    out = np.empty((sv.n, 16))
    lib().or_segment_details(C.byref(cfg.c), C.byref(sv.c), _p(out))
    return {f: out[:, i] for i, f in enumerate(SEG_FIELDS)}


def lookup(cfg: Config, h) -> np.ndarray:
    """(m, 6): psi, P1..P5 at altitudes h."""
    h = np.ascontiguousarray(np.atleast_1d(h), dtype=np.float64)
    out = np.empty((h.shape[0], 6))
    lib().or_lookup_many(C.byref(cfg.c), h.shape[0], _p(h), _p(out))
    return out


PROP_FIELDS = ("x_g", "y_g", "T", "u_o", "v_o", "w_o", "n_e", "psi_e", "S")


def propagate(cfg: Config, x_e, y_e, h_e, u, v, w) -> dict:
    inp = np.ascontiguousarray(np.stack(np.broadcast_arrays(
        *[np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (x_e, y_e, h_e, u, v, w)]),
        axis=1))
    out = np.empty((inp.shape[0], 9))
    lib().or_propagate_many(C.byref(cfg.c), inp.shape[0], _p(inp), _p(out))
    return {f: out[:, i] for i, f in enumerate(PROP_FIELDS)}


def propagate_exact(cfg: Config, x_e, y_e, h_e, u, v, w) -> dict:
    """Cell-by-cell exact propagation (the slow path for grazing bunches)."""
    inp = np.ascontiguousarray(np.stack(np.broadcast_arrays(
        *[np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (x_e, y_e, h_e, u, v, w)]),
        axis=1))
    out = np.empty((inp.shape[0], 9))
    lib().or_propagate_exact_many(C.byref(cfg.c), inp.shape[0], _p(inp), _p(out))
    return {f: out[:, i] for i, f in enumerate(PROP_FIELDS)}


def propagate_curved(cfg: Config, x_e, y_e, z_e, u, v, w) -> dict:
    """Exact propagation through spherical shells of radius cfg.earth_radius
    (the curved variant); (x_e, y_e, z_e) Cartesian with z along the array
    origin's vertical.  Adds 'status' (-1 reached the ground, else the drop
    reason index: upward or grazing)."""
    if not cfg.earth_radius > 0.0:
        raise ValueError("propagate_curved needs earth_radius > 0")
    inp = np.ascontiguousarray(np.stack(np.broadcast_arrays(
        *[np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (x_e, y_e, z_e, u, v, w)]),
        axis=1))
    out = np.empty((inp.shape[0], 10))
    lib().or_propagate_curved_many(C.byref(cfg.c), inp.shape[0], _p(inp), _p(out))
    d = {f: out[:, i + 1] for i, f in enumerate(PROP_FIELDS)}
    d["status"] = out[:, 0].astype(np.int64)
    return d


def curved_altitude(R: float, x: float, y: float, z: float) -> float:
    return lib().or_curved_altitude(float(R), float(x), float(y), float(z))


def philox(ctr, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(ctr), _p(key), _p(out))
    return out


def sphere_disc(x_g, y_g, u_o, v_o, X, Y, R) -> float:
    return lib().or_sphere_disc(x_g, y_g, u_o, v_o, X, Y, R)


def frank_tamm_k(lambda_min=300.0, lambda_max=600.0) -> float:
    return lib().or_frank_tamm_k(lambda_min, lambda_max)


# ---------------------------------------------------------------------------
# differentiation pattern: parameterised atmosphere and soft telescope response
# ---------------------------------------------------------------------------

@dataclass
class AtmoParamSpec:
    """log eta(h) = log eta0 - int_0^h dh'/H(h') + Lambda(h).

    H is constant inside each layer [bounds[l], bounds[l+1]) (the last layer
    extends upward); Lambda interpolates knot values linearly at
    h_j = j * knot_top / (n_knots - 1) and is constant above knot_top."""
    eta0: float
    layer_bounds: np.ndarray     # n_layers + 1, starting at 0
    n_knots: int
    knot_top: float
    obs_level: float
    step: float
    top: float

    @property
    def n_layers(self) -> int:
        return len(self.layer_bounds) - 1

    def grid(self) -> np.ndarray:
        n = int(np.floor((self.top - self.obs_level) / self.step)) + 1
        return self.obs_level + np.arange(n) * self.step


def eta_from_params(spec: AtmoParamSpec, theta, h) -> np.ndarray:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    assert theta.shape[0] == spec.n_knots + spec.n_layers
    h = np.ascontiguousarray(np.atleast_1d(h), dtype=np.float64)
    b = np.ascontiguousarray(spec.layer_bounds, dtype=np.float64)
    out = np.empty_like(h)
    lib().or_eta_param_many(spec.eta0, spec.n_layers, _p(b), spec.n_knots, spec.knot_top,
                            _p(theta), h.shape[0], _p(h), _p(out))
    return out


def tables_from_params(spec: AtmoParamSpec, theta) -> Tables:
    """Tables of the parameterised profile sampled at the grid nodes."""
    g = spec.grid()
    return build_tables(g, eta_from_params(spec, theta, g), spec.obs_level, spec.step)


def soft(cfg: Config, segs, n_b_frozen, sigma: float, nthreads: int = 1, seg_id_base=None,
         seg_id=None):
    """(S, A), each (n_showers, n_tel): soft photon counts and photon-weighted times.
    seg_id_base / seg_id as in run()."""
    if cfg.earth_radius > 0.0:
        raise ValueError("the soft response is defined for the plane-parallel atmosphere")
    sv = SegView(segs, seg_id_base=seg_id_base, seg_id=seg_id)
    nb = np.ascontiguousarray(n_b_frozen, dtype=np.int64)
    S = np.zeros(sv.n_showers * cfg.n_tel)
    A = np.zeros(sv.n_showers * cfg.n_tel)
    lib().or_soft(C.byref(cfg.c), C.byref(sv.c), _p(nb), float(sigma), sv.n_showers,
                  int(nthreads), _p(S), _p(A))
    return S.reshape(sv.n_showers, cfg.n_tel), A.reshape(sv.n_showers, cfg.n_tel)
