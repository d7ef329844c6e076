"""Python binding of libckv.so (ctypes): argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch supplies device
memory and the stream.  Importing this module does not load the library;
the first call does, and raises if `libckv.so` has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libckv.so")

CKV_FP64 = 0
CKV_MIXED = 1
DROP_NAMES = ("mass", "threshold", "nonfinite", "below_obs", "above_top", "upward", "grazing")
RECORD_FIELDS = ("dx", "dy", "u_obs", "v_obs", "t", "h_emit", "photons", "lambda")

EXPORTED = ("ckv_last_error", "ckv_version", "ckv_atmo_create", "ckv_atmo_info", "ckv_atmo_tables",
            "ckv_atmo_destroy", "ckv_array_create", "ckv_array_destroy", "ckv_workspace_size",
            "ckv_run", "ckv_count", "ckv_atmo_from_params", "ckv_atmo_params_backward",
            "ckv_array_create_soft", "ckv_soft_forward", "ckv_soft_backward",
            "ckv_atmo_create_with_depth", "ckv_atmo_depth", "ckv_profile_bins",
            "ckv_atmo_create_nodes", "ckv_atmo_nodes", "ckv_run_noalloc",
            "ckv_noalloc_workspace_size")


class CkvError(RuntimeError):
    pass


class _Segments(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x0", "y0", "h0", "u", "v", "w", "length", "t0",
                                          "energy", "ptype")] + [("n", C.c_int64),
                                                                 ("step_id", C.c_void_p)]


class _Showers(C.Structure):
    _fields_ = [("seg_offsets", C.c_void_p), ("t_ref", C.c_void_p), ("shower_ids", C.c_void_p),
                ("seg_id_base", C.c_void_p), ("n_showers", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("bunch_size", C.c_double), ("lambda_min_nm", C.c_double),
                ("lambda_max_nm", C.c_double), ("w_min", C.c_double), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("tile_segments", C.c_int32), ("grid", C.c_int32),
                ("waves_per_group", C.c_int32), ("event_begin", C.c_void_p),
                ("event_end", C.c_void_p), ("depth_bin_gcm2", C.c_double),
                ("grazing_exact", C.c_int32), ("reserved", C.c_int32),
                ("earth_radius_m", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("n_bunches", C.c_int64), ("n_hits", C.c_int64), ("n_records", C.c_int64),
                ("n_emitting", C.c_int64), ("n_tiles", C.c_int64), ("drops", C.c_int64 * 8),
                ("resume_step", C.c_int64), ("resume_shower", C.c_int32),
                ("overflow", C.c_int32), ("error", C.c_int32), ("reserved", C.c_int32)]


class _Cursor(C.Structure):
    _fields_ = [("step", C.c_int64), ("shower", C.c_int32), ("reserved", C.c_int32)]


class _ParamSpec(C.Structure):
    _fields_ = [("eta0", C.c_double), ("n_layers", C.c_int32), ("n_knots", C.c_int32),
                ("layer_bounds_m", C.c_void_p), ("knot_top_m", C.c_double),
                ("obs_level_m", C.c_double), ("step_m", C.c_double), ("top_m", C.c_double)]


class _SoftList(C.Structure):
    _fields_ = [("ids", C.c_void_p), ("capacity", C.c_int64), ("count", C.c_void_p)]


class _Output(C.Structure):
    _fields_ = [("records", C.c_void_p), ("ids", C.c_void_p), ("capacity", C.c_int64),
                ("tel_offsets", C.c_void_p), ("result", C.c_void_p),
                ("profile_photons", C.c_void_p), ("profile_bunches", C.c_void_p)]


RESULT_BYTES = C.sizeof(_Result)
_lib = None


def lib():
    """The loaded library; raises CkvError if it was not built, or was built from
    other sources than the ones beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CkvError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        from . import build as _build
        have, want = _build.built_hash(), _build.source_hash()
        if have != want:
            raise CkvError(f"{LIB_PATH} was built from other sources (built {have}, sources {want}): "
                           "rebuild it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ckv_last_error.restype = C.c_char_p
        L.ckv_version.restype = C.c_int
        L.ckv_atmo_create.argtypes = [P, P, I64, D, D, C.POINTER(P)]
        L.ckv_atmo_create_with_depth.argtypes = [P, P, P, I64, D, D, C.POINTER(P)]
        L.ckv_atmo_depth.argtypes = [P, P]
        L.ckv_profile_bins.argtypes = [P, D, P]
        L.ckv_atmo_create_nodes.argtypes = [P, P, I64, D, C.POINTER(P)]
        L.ckv_atmo_nodes.argtypes = [P, P]
        L.ckv_atmo_info.argtypes = [P, P, P, P]
        L.ckv_atmo_tables.argtypes = [P, P, P]
        L.ckv_atmo_destroy.argtypes = [P]
        L.ckv_array_create.argtypes = [P, P, P, I32, C.POINTER(P)]
        L.ckv_array_destroy.argtypes = [P]
        L.ckv_workspace_size.restype = C.c_size_t
        L.ckv_workspace_size.argtypes = [I64, I32, I32, I64, C.POINTER(_Params)]
        L.ckv_run.argtypes = [C.POINTER(_Segments), C.POINTER(_Showers), C.POINTER(_Params), P, P,
                              P, C.c_size_t, C.POINTER(_Output), C.POINTER(_Cursor), P]
        L.ckv_count.argtypes = [C.POINTER(_Segments), C.POINTER(_Params), P, P, P]
        L.ckv_run_noalloc.argtypes = [C.POINTER(_Segments), C.POINTER(_Showers), C.POINTER(_Params),
                                      P, P, C.POINTER(_Output), C.POINTER(_Cursor), P]
        L.ckv_noalloc_workspace_size.restype = C.c_size_t
        L.ckv_noalloc_workspace_size.argtypes = [I64, I32, I32, I64, C.POINTER(_Params)]
        L.ckv_atmo_from_params.argtypes = [C.POINTER(_ParamSpec), P, C.POINTER(P)]
        L.ckv_atmo_params_backward.argtypes = [C.POINTER(_ParamSpec), P, P, P, P, P]
        L.ckv_array_create_soft.argtypes = [P, P, P, I32, D, C.POINTER(P)]
        L.ckv_soft_forward.argtypes = [C.POINTER(_Segments), C.POINTER(_Showers), C.POINTER(_Params),
                                       P, P, P, P, P, C.POINTER(_SoftList), P, P, C.c_size_t, P]
        L.ckv_soft_backward.argtypes = [C.POINTER(_Segments), C.POINTER(_Showers), C.POINTER(_Params),
                                        P, P, P, P, P, P, P, C.POINTER(_SoftList), P, P, C.c_size_t,
                                        P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise CkvError(f"ckv error {rc}: {lib().ckv_last_error().decode()}")


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Atmosphere:
    """ckv_atmo: uniform fine tables built from a tabulated n-1 profile."""

    def __init__(self, alt=None, eta=None, obs_level: float = 0.0, step: float = 0.0, handle=None,
                 depth=None, nodes: bool = False):
        """nodes=True: tables on the profile's own altitudes, binary-search lookups."""
        self._L = lib()
        if handle is not None:          # adopt a handle made by another constructor
            self.handle = handle
            return
        self._alt = np.ascontiguousarray(alt, dtype=np.float64)
        self._eta = np.ascontiguousarray(eta, dtype=np.float64)
        h = C.c_void_p()
        if nodes:
            _check(lib().ckv_atmo_create_nodes(_np_ptr(self._alt), _np_ptr(self._eta),
                                               self._alt.shape[0], float(obs_level), C.byref(h)))
        elif depth is None:
            _check(lib().ckv_atmo_create(_np_ptr(self._alt), _np_ptr(self._eta), self._alt.shape[0],
                                         float(obs_level), float(step), C.byref(h)))
        else:
            self._depth = np.ascontiguousarray(depth, dtype=np.float64)
            _check(lib().ckv_atmo_create_with_depth(_np_ptr(self._alt), _np_ptr(self._eta),
                                                    _np_ptr(self._depth), self._alt.shape[0],
                                                    float(obs_level), float(step), C.byref(h)))
        self.handle = h

    def nodes(self) -> np.ndarray:
        """Node altitudes [m]."""
        n, _, _ = self.info()
        out = np.empty(n)
        _check(lib().ckv_atmo_nodes(self.handle, _np_ptr(out)))
        return out

    def depth(self) -> np.ndarray:
        """Vertical depth [g/cm^2] at the grid nodes."""
        n, _, _ = self.info()
        out = np.empty(n)
        _check(lib().ckv_atmo_depth(self.handle, _np_ptr(out)))
        return out

    def profile_bins(self, width_gcm2: float) -> int:
        nb = C.c_int32()
        _check(lib().ckv_profile_bins(self.handle, float(width_gcm2), C.byref(nb)))
        return nb.value

    def info(self):
        n = C.c_int64()
        h = C.c_double()
        st = C.c_double()
        _check(lib().ckv_atmo_info(self.handle, C.byref(n), C.byref(h), C.byref(st)))
        return n.value, h.value, st.value

    def tables(self):
        n, _, _ = self.info()
        psi = np.empty(n)
        P = np.empty((5, n))
        _check(lib().ckv_atmo_tables(self.handle, _np_ptr(psi), _np_ptr(P)))
        return psi, P

    def close(self):
        # the library is held by the object: module globals may be gone at exit
        L = getattr(self, "_L", None)
        if getattr(self, "handle", None) and L is not None:
            L.ckv_atmo_destroy(self.handle)
            self.handle = None

    __del__ = close


class TelescopeArray:
    """ckv_array: telescope spheres and their candidate grid (and, with
    soft_sigma > 0, the grid of the soft response)."""

    def __init__(self, x, y, r, soft_sigma: float = 0.0):
        self._L = lib()
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.r = np.ascontiguousarray(r, dtype=np.float64)
        self.soft_sigma = float(soft_sigma)
        h = C.c_void_p()
        if soft_sigma > 0:
            _check(lib().ckv_array_create_soft(_np_ptr(self.x), _np_ptr(self.y), _np_ptr(self.r),
                                               self.x.shape[0], self.soft_sigma, C.byref(h)))
        else:
            _check(lib().ckv_array_create(_np_ptr(self.x), _np_ptr(self.y), _np_ptr(self.r),
                                          self.x.shape[0], C.byref(h)))
        self.handle = h

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def close(self):
        L = getattr(self, "_L", None)
        if getattr(self, "handle", None) and L is not None:
            L.ckv_array_destroy(self.handle)
            self.handle = None

    __del__ = close


# ---------------------------------------------------------------------------
# device inputs
# ---------------------------------------------------------------------------

class DeviceSegments:
    """Segments and shower bookkeeping resident in device memory (torch)."""

    FIELDS = ("x0", "y0", "h0", "u", "v", "w", "length", "t0", "energy")

    def __init__(self, segs, device="cuda", seg_id_base=None, step_id=None):
        """step_id (optional, one uint32 per step): the random-number counter word of
        each step, so that reordered steps keep their bunches."""
        import torch
        self.t = {f: torch.as_tensor(np.ascontiguousarray(getattr(segs, f), dtype=np.float64),
                                     device=device) for f in self.FIELDS}
        self.t["ptype"] = torch.as_tensor(np.ascontiguousarray(segs.ptype, dtype=np.uint8),
                                          device=device)
        self.seg_offsets = torch.as_tensor(np.asarray(segs.seg_offsets, dtype=np.int64), device=device)
        self.t_ref = torch.as_tensor(np.asarray(segs.t_ref, dtype=np.float64), device=device)
        self.shower_ids = torch.as_tensor(np.asarray(segs.shower_ids, dtype=np.uint32).view(np.int32),
                                          device=device)
        self.seg_id_base = None if seg_id_base is None else torch.as_tensor(
            np.asarray(seg_id_base, dtype=np.int64), device=device)
        self.step_id = None if step_id is None else torch.as_tensor(
            np.ascontiguousarray(step_id, dtype=np.uint32).view(np.int32), device=device)
        self.n = segs.n
        self.n_showers = segs.n_showers
        self.offsets_host = np.asarray(segs.seg_offsets, dtype=np.int64).copy()
        self.base_host = (np.zeros(self.n_showers, dtype=np.int64) if seg_id_base is None
                          else np.asarray(seg_id_base, dtype=np.int64).copy())

    def view(self, a: int, b: int) -> "DeviceSegments":
        """Steps [a, b) as their own input, without copying the step arrays: the
        showers they touch keep their ids and t_ref, and each shower's first step
        in the range keeps its step index (seg_id_base), so every bunch keeps its
        random numbers."""
        import torch
        off = self.offsets_host
        s0 = int(np.searchsorted(off, a, side="right") - 1)
        s1 = int(np.searchsorted(off, b, side="left"))          # exclusive
        s1 = max(s1, s0 + 1)
        v = DeviceSegments.__new__(DeviceSegments)
        v.t = {f: t[a:b] for f, t in self.t.items()}
        v.step_id = None if self.step_id is None else self.step_id[a:b]
        sub_off = np.clip(off[s0:s1 + 1], a, b) - a
        sub_off[0], sub_off[-1] = 0, b - a
        dev = self.t["x0"].device
        v.seg_offsets = torch.as_tensor(sub_off, device=dev)
        v.t_ref = self.t_ref[s0:s1]
        v.shower_ids = self.shower_ids[s0:s1]
        base = self.base_host[s0:s1] + np.maximum(a - off[s0:s1], 0)
        v.seg_id_base = torch.as_tensor(base, device=dev)
        v.n, v.n_showers = b - a, s1 - s0
        v.offsets_host, v.base_host = sub_off, base
        v.shower_range = (s0, s1)
        return v

    def c_segments(self) -> _Segments:
        t = self.t
        return _Segments(*[t[f].data_ptr() for f in self.FIELDS], t["ptype"].data_ptr(), self.n,
                         self.step_id.data_ptr() if self.step_id is not None else None)

    def c_showers(self) -> _Showers:
        return _Showers(self.seg_offsets.data_ptr(), self.t_ref.data_ptr(),
                        self.shower_ids.data_ptr(),
                        self.seg_id_base.data_ptr() if self.seg_id_base is not None else None,
                        self.n_showers)


def make_params(*, precision=CKV_MIXED, bunch_size=5.0, lambda_min=300.0, lambda_max=600.0,
                w_min=0.1, seed=0x14927, tile_segments=0, grid=0, waves_per_group=0,
                event_begin=None, event_end=None, depth_bin=0.0, grazing_exact=False,
                earth_radius=0.0) -> _Params:
    """depth_bin > 0 [g/cm^2]: also the longitudinal photon-production profile;
    grazing_exact: trace bunches with 0 < w <= w_min exactly instead of dropping them;
    earth_radius > 0 [m]: curved atmosphere (spherical shells), every bunch traced exactly."""
    return _Params(bunch_size, lambda_min, lambda_max, w_min, int(seed) & (2**64 - 1),
                   int(precision), int(tile_segments), int(grid), int(waves_per_group),
                   event_begin, event_end, float(depth_bin), int(bool(grazing_exact)), 0,
                   float(earth_radius))


def workspace_size(n_segments, n_showers, n_tel, capacity, params: _Params) -> int:
    return int(lib().ckv_workspace_size(n_segments, n_showers, n_tel, capacity, C.byref(params)))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class RunOutput:
    records: "object"       # torch float32 (capacity, 8)
    ids: "object"           # torch int64 (capacity, 2) or None
    tel_offsets: "object"   # torch int64 (n_showers*n_tel + 1)
    result_raw: "object"    # torch uint8 (RESULT_BYTES)
    profile_photons: "object" = None   # torch float64 (n_showers, n_bins) or None
    profile_bunches: "object" = None   # torch int64 (n_showers, n_bins) or None

    def result(self) -> dict:
        r = _Result.from_buffer_copy(self.result_raw.cpu().numpy().tobytes())
        return dict(n_bunches=r.n_bunches, n_hits=r.n_hits, n_records=r.n_records,
                    n_emitting=r.n_emitting, n_tiles=r.n_tiles,
                    drops=dict(zip(DROP_NAMES, list(r.drops)[:7])), overflow=r.overflow,
                    error=r.error, resume_step=r.resume_step, resume_shower=r.resume_shower)


class Runner:
    """Holds the workspace and outputs for repeated ckv_run calls of one shape."""

    def __init__(self, dsegs: DeviceSegments, atmo: Atmosphere, tels: TelescopeArray,
                 params: _Params, capacity: int, want_ids: bool = True, device="cuda"):
        import torch
        self.dsegs, self.atmo, self.tels, self.params = dsegs, atmo, tels, params
        self.capacity = int(capacity)
        ws = workspace_size(dsegs.n, dsegs.n_showers, tels.n, self.capacity, params)
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        self.records = torch.empty((max(self.capacity, 1), 8), dtype=torch.float32, device=device)
        self.ids = torch.empty((max(self.capacity, 1), 2), dtype=torch.int64, device=device) \
            if want_ids else None
        self.tel_offsets = torch.empty(dsegs.n_showers * tels.n + 1, dtype=torch.int64, device=device)
        self.result_raw = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)
        self.profile_photons = self.profile_bunches = None
        if params.depth_bin_gcm2 > 0:
            nb = atmo.profile_bins(params.depth_bin_gcm2)
            self.profile_photons = torch.empty((dsegs.n_showers, nb), dtype=torch.float64, device=device)
            self.profile_bunches = torch.empty((dsegs.n_showers, nb), dtype=torch.int64, device=device)
        self._segs = dsegs.c_segments()
        self._showers = dsegs.c_showers()
        self._out = _Output(self.records.data_ptr(),
                            self.ids.data_ptr() if self.ids is not None else None,
                            self.capacity, self.tel_offsets.data_ptr(), self.result_raw.data_ptr(),
                            self.profile_photons.data_ptr() if self.profile_photons is not None else None,
                            self.profile_bunches.data_ptr() if self.profile_bunches is not None else None)

    def run(self, stream=None, resume_from=None) -> RunOutput:
        """resume_from: (step, shower) where to start, e.g. the resume_step and
        resume_shower of a run that overflowed; None = the first step."""
        cur = None if resume_from is None else C.byref(_Cursor(int(resume_from[0]),
                                                               int(resume_from[1]), 0))
        _check(lib().ckv_run(C.byref(self._segs), C.byref(self._showers), C.byref(self.params),
                             self.atmo.handle, self.tels.handle, C.c_void_p(self.workspace.data_ptr()),
                             self.workspace.numel(), C.byref(self._out), cur, _stream_ptr(stream)))
        return RunOutput(self.records, self.ids, self.tel_offsets, self.result_raw,
                         self.profile_photons, self.profile_bunches)


def count(dsegs: DeviceSegments, atmo: Atmosphere, params: _Params, stream=None):
    """Bunches per step (device int64 tensor)."""
    import torch
    n_b = torch.empty(max(dsegs.n, 1), dtype=torch.int64, device=dsegs.t["x0"].device)
    segs = dsegs.c_segments()
    _check(lib().ckv_count(C.byref(segs), C.byref(params), atmo.handle,
                           C.c_void_p(n_b.data_ptr()), _stream_ptr(stream)))
    return n_b[:dsegs.n]


def run(segs, atmo: Atmosphere, tels: TelescopeArray, *, capacity: int, want_ids=True,
        stream=None, **param_kw) -> RunOutput:
    """One-shot convenience: segments (synth.Segments or DeviceSegments) -> records."""
    d = segs if isinstance(segs, DeviceSegments) else DeviceSegments(segs)
    return Runner(d, atmo, tels, make_params(**param_kw), capacity, want_ids).run(stream)


@dataclass
class Chunk:
    """One range of a streamed run: steps [begin, end) of the input, showers
    [shower_begin, shower_end), and its n_records records grouped per
    (shower, telescope) through tel_offsets."""
    begin: int
    end: int
    shower_begin: int
    shower_end: int
    records: "object"
    ids: "object"
    tel_offsets: "object"
    result: dict


class _OutBuf:
    """Device output of one ckv_run: records, ids, CSR offsets, result."""

    def __init__(self, capacity: int, n_groups: int, want_ids: bool, device):
        import torch
        self.records = torch.empty((max(capacity, 1), 8), dtype=torch.float32, device=device)
        self.ids = torch.empty((max(capacity, 1), 2), dtype=torch.int64, device=device) \
            if want_ids else None
        self.tel_offsets = torch.empty(n_groups + 1, dtype=torch.int64, device=device)
        self.result_raw = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)

    def c_output(self, capacity: int) -> _Output:
        return _Output(self.records.data_ptr(), self.ids.data_ptr() if self.ids is not None else None,
                       capacity, self.tel_offsets.data_ptr(), self.result_raw.data_ptr())

    def result(self) -> dict:
        return RunOutput(self.records, self.ids, self.tel_offsets, self.result_raw).result()


class Streamer:
    """ckv_run over consecutive step ranges of a large input, each sized so that
    its records fit one output chunk (8 388 608 records = 256 MB by default).

    Ranges are planned from the bunch counts of the steps (ckv_count, summed on
    the device into one prefix value per block of `plan_block` steps) and the
    largest crossings-per-bunch ratio seen so far.  A range whose crossings do
    not fit the chunk writes a complete prefix of its steps (ckv_run's resume
    cursor): that prefix becomes the chunk and the next range starts where it
    ended, so no step is computed for output twice unless a single tile of
    steps alone exceeds the chunk.  Per (shower, telescope), the records of
    consecutive chunks concatenate in the one-shot (step, bunch) order.

    chunks() yields each range's output on the device; to_host() copies every
    chunk to pinned host memory while the next range is computed."""

    def __init__(self, dsegs: DeviceSegments, atmo: Atmosphere, tels: TelescopeArray,
                 params: _Params, chunk_records: int = 8_388_608, want_ids: bool = True,
                 first_ratio: float = 0.05, max_range: Optional[int] = None,
                 plan_block: int = 4096, device="cuda"):
        import torch
        if params.depth_bin_gcm2 > 0:
            raise CkvError("Streamer: run the longitudinal profile with Runner (one launch)")
        self.dsegs, self.atmo, self.tels, self.params = dsegs, atmo, tels, params
        self.capacity = int(chunk_records)
        self.want_ids = want_ids
        self.device = device
        n = dsegs.n
        self.block = int(plan_block)
        n_b = count(dsegs, atmo, params)
        cum = torch.cumsum(n_b, 0)
        self._cum = cum                     # device: bunches of steps [0, i]
        ends = torch.arange(self.block, n + self.block, self.block, device=cum.device).clamp_(max=n)
        self.plan_at = np.concatenate([[0], ends.cpu().numpy()]).astype(np.int64)
        self.plan_cum = np.zeros(len(self.plan_at), dtype=np.int64)
        if n:
            self.plan_cum[1:] = cum[ends - 1].cpu().numpy()
        self.ratio = float(first_ratio)     # crossings per bunch assumed for planning
        self.max_seen = 0.0
        self.max_range = n if max_range is None else int(max_range)
        ws = workspace_size(max(self.max_range, 1), dsegs.n_showers, tels.n, self.capacity, params)
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        self.out = _OutBuf(self.capacity, dsegs.n_showers * tels.n, want_ids, device)
        self.n_reruns = 0        # ranges computed again because nothing of them fit
        self.n_resumed = 0       # ranges cut short at a resume cursor

    @property
    def total_bunches(self) -> int:
        return int(self.plan_cum[-1])

    def bunches(self, a: int, b: int) -> int:
        """Bunches of steps [a, b) (from the plan's counts; synchronises)."""
        if b <= a:
            return 0
        hi = int(self._cum[b - 1].item())
        return hi - (int(self._cum[a - 1].item()) if a > 0 else 0)

    def _cum_at(self, x: int) -> float:
        return float(np.interp(x, self.plan_at, self.plan_cum))

    def _range_end(self, a: int) -> int:
        budget = 0.8 * self.capacity / max(self.ratio, 1e-12)
        target = self._cum_at(a) + budget
        j = int(np.searchsorted(self.plan_cum, target, side="right")) - 1
        b = int(self.plan_at[max(j, 0)])
        if b <= a:                          # less than one block fits: interpolate inside it
            b = int(np.interp(target, self.plan_cum, self.plan_at))
        return int(min(max(b, a + 1), self.dsegs.n, a + self.max_range))

    def _launch(self, a: int, b: int, out: _OutBuf, stream=None):
        v = self.dsegs.view(a, b)
        segs, showers, o = v.c_segments(), v.c_showers(), out.c_output(self.capacity)
        _check(lib().ckv_run(C.byref(segs), C.byref(showers), C.byref(self.params), self.atmo.handle,
                             self.tels.handle, C.c_void_p(self.workspace.data_ptr()),
                             self.workspace.numel(), C.byref(o), None, _stream_ptr(stream)))
        return v

    def _accept(self, a: int, b: int, res: dict) -> int:
        """Updates the planning ratio; returns the end of the written part of range
        [a, b) (a when nothing of it fit and it has to be run again, smaller)."""
        if res["error"]:
            raise CkvError(f"device reported error flags {res['error']} on steps [{a}, {b})")
        seen = res["n_hits"] / max(res["n_bunches"], 1)
        if res["overflow"]:
            self.max_seen = max(self.max_seen, seen * 1.25)
            self.ratio = self.max_seen
            end = a + int(res["resume_step"])
            if end <= a:
                if b == a + 1:
                    raise CkvError(f"step {a} alone has {res['n_hits']} crossings > chunk capacity")
                self.n_reruns += 1
            else:
                self.n_resumed += 1
            return end
        self.max_seen = max(self.max_seen, seen)
        if self.max_seen > 0:
            self.ratio = 1.1 * self.max_seen
        return b

    def chunks(self, stream=None):
        """Yields Chunk objects (device buffers, reused by the next chunk) in step order."""
        import torch
        a, n = 0, self.dsegs.n
        while a < n:
            b = self._range_end(a)
            v = self._launch(a, b, self.out, stream)
            torch.cuda.synchronize()
            res = self.out.result()
            end = self._accept(a, b, res)
            if end <= a:
                continue
            k = int(res["n_records"])
            yield Chunk(a, end, *v.shower_range, self.out.records[:k],
                        self.out.ids[:k] if self.out.ids is not None else None,
                        self.out.tel_offsets[:v.n_showers * self.tels.n + 1], res)
            a = end

    def to_host(self, sink):
        """Streams every chunk to pinned host memory: sink(chunk) receives a Chunk
        whose records, ids and tel_offsets are host tensors (valid during the
        call).  The device-to-host copy of a chunk runs on its own stream while
        the next range is computed into a second output buffer."""
        import torch
        comp = torch.cuda.current_stream()
        copy = torch.cuda.Stream()
        outs = [self.out, _OutBuf(self.capacity, self.dsegs.n_showers * self.tels.n, self.want_ids,
                                  self.device)]
        n_groups = self.dsegs.n_showers * self.tels.n + 1
        host = [dict(records=torch.empty((self.capacity, 8), dtype=torch.float32, pin_memory=True),
                     ids=torch.empty((self.capacity, 2), dtype=torch.int64, pin_memory=True)
                     if self.want_ids else None,
                     off=torch.empty(n_groups, dtype=torch.int64, pin_memory=True))
                for _ in range(2)]
        copied = [None, None]          # event: copy out of buffer i finished
        pending = None

        def deliver(p):
            ev, slot, meta = p
            ev.synchronize()
            h = host[slot]
            k = int(meta["res"]["n_records"])
            sink(Chunk(meta["a"], meta["b"], *meta["showers"], h["records"][:k],
                       h["ids"][:k] if h["ids"] is not None else None, h["off"][:meta["ng"]],
                       meta["res"]))

        a, n, i = 0, self.dsegs.n, 0
        while a < n:
            b = self._range_end(a)
            slot = i % 2
            out = outs[slot]
            if copied[slot] is not None:
                comp.wait_event(copied[slot])      # its last copy must be done before reuse
            v = self._launch(a, b, out, comp)
            ran = torch.cuda.Event()
            ran.record(comp)
            if pending is not None:                # hand over the previous chunk meanwhile
                deliver(pending)
                pending = None
            ran.synchronize()
            res = out.result()
            end = self._accept(a, b, res)
            if end <= a:
                continue
            k = int(res["n_records"])
            ng = v.n_showers * self.tels.n + 1
            copy.wait_event(ran)
            with torch.cuda.stream(copy):
                h = host[slot]
                h["records"][:k].copy_(out.records[:k], non_blocking=True)
                if h["ids"] is not None:
                    h["ids"][:k].copy_(out.ids[:k], non_blocking=True)
                h["off"][:ng].copy_(out.tel_offsets[:ng], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(copy)
            copied[slot] = ev
            pending = (ev, slot, dict(a=a, b=end, showers=v.shower_range, res=res, ng=ng))
            a, i = end, i + 1
        if pending is not None:
            deliver(pending)
        torch.cuda.synchronize()


class GraphRunner:
    """A Runner's ckv_run captured once into a HIP graph and replayed.

    ckv_run enqueues kernels only (no allocation, copy or memset), so the whole
    bunch path is one graph; one eager run first sets the kernels' launch
    attributes outside the capture."""

    def __init__(self, runner: Runner):
        import torch
        self.runner = runner
        runner.run()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        self.stream = torch.cuda.Stream()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self.out = runner.run()

    def replay(self) -> RunOutput:
        self.graph.replay()
        return self.out



# ---------------------------------------------------------------------------
# differentiation: soft telescope response and its gradient
# ---------------------------------------------------------------------------

class ParamSpec:
    """ckv_atmo_param_spec (see include/ckv.h)."""

    def __init__(self, eta0, layer_bounds, n_knots, knot_top, obs_level, step, top):
        self.bounds = np.ascontiguousarray(layer_bounds, dtype=np.float64)
        self.c = _ParamSpec(float(eta0), self.bounds.shape[0] - 1, int(n_knots),
                            _np_ptr(self.bounds).value, float(knot_top), float(obs_level),
                            float(step), float(top))

    @property
    def n_theta(self) -> int:
        return self.c.n_knots + self.c.n_layers

    def atmosphere(self, theta) -> Atmosphere:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().ckv_atmo_from_params(C.byref(self.c), _np_ptr(th), C.byref(h)))
        return Atmosphere(handle=h)

    def backward(self, theta, atmo: Atmosphere, g_psi, g_P) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        gp = np.ascontiguousarray(g_psi, dtype=np.float64)
        gq = np.ascontiguousarray(g_P, dtype=np.float64)
        out = np.empty(self.n_theta)
        _check(lib().ckv_atmo_params_backward(C.byref(self.c), _np_ptr(th), atmo.handle,
                                              _np_ptr(gp), _np_ptr(gq), _np_ptr(out)))
        return out


class SoftModel:
    """theta -> (S, A) per (shower, telescope), with bunch counts frozen at theta0.

    With use_list (default) the forward records the bunches that have a nonzero
    weight and the backward at the same theta recomputes only those; the list
    grows after a backward that found it too small (that backward, and any at
    another theta, recompute every bunch)."""

    def __init__(self, segs, tels, spec: ParamSpec, theta0, sigma: float, *, bunch_size=5.0,
                 lambda_min=300.0, lambda_max=600.0, seed=0x14927, device="cuda",
                 use_list=True, list_capacity=None):
        import torch
        self.spec = spec
        self.dsegs = segs if isinstance(segs, DeviceSegments) else DeviceSegments(segs, device=device)
        self.tels = TelescopeArray(tels.x, tels.y, tels.r, soft_sigma=sigma)
        self.params = make_params(precision=CKV_FP64, bunch_size=bunch_size, lambda_min=lambda_min,
                                  lambda_max=lambda_max, seed=seed)
        self.atmo0 = spec.atmosphere(theta0)
        self.n_b = count(self.dsegs, self.atmo0, self.params).contiguous()
        ws = workspace_size(self.dsegs.n, self.dsegs.n_showers, self.tels.n, 0, self.params)
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        n_nodes = self.atmo0.info()[0]
        # dL/dpsi and dL/dP side by side: the backward brings both to the host in one copy
        self._g = torch.empty(6 * n_nodes, dtype=torch.float64, device=device)
        self.g_psi, self.g_P = self._g[:n_nodes], self._g[n_nodes:]
        self.shape = (self.dsegs.n_showers, self.tels.n)
        self._segs = self.dsegs.c_segments()
        self._showers = self.dsegs.c_showers()
        self._cache = None
        self.use_list = bool(use_list)
        self.list_count = torch.zeros(1, dtype=torch.int64, device=device)
        self.result_raw = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)
        self._list_theta = None
        if self.use_list:
            cap = list_capacity if list_capacity is not None else int(self.n_b.sum()) // 8 + 1024
            self._alloc_list(int(cap))
        # The conditions the soft kernels report (bad shower offsets; a 32-step tile
        # with 2^30 or more frozen bunches) depend on the segments and the frozen
        # counts only, not on theta: a tile's bunches at any theta are some of its
        # steps' frozen counts, and a tile lies inside some window of 32 consecutive
        # steps.  When no such window holds 2^30, one clean pass of each kind proves
        # every later one clean, and those skip the check and its synchronisation.
        cs = torch.cumsum(self.n_b, 0)
        if cs.numel() > 32:
            cs = torch.cat([cs[31:32], cs[32:] - cs[:-32]])
        self._bound_holds = bool(cs.numel() == 0 or int(cs.max()) < (1 << 30))
        self._clean = {"forward": False, "backward": False}

    def _alloc_list(self, capacity: int):
        import torch
        self.list_ids = torch.empty(max(capacity, 1), dtype=torch.int64, device=self.g_psi.device)
        self._list = _SoftList(self.list_ids.data_ptr(), int(capacity), self.list_count.data_ptr())
        self._list_theta = None

    def list_state(self):
        """(ids found by the last forward, capacity); synchronises."""
        return int(self.list_count.item()), int(self._list.capacity) if self.use_list else 0

    def _atmo(self, theta):
        th = np.asarray(theta, dtype=np.float64)
        if self._cache is None or not np.array_equal(self._cache[0], th):
            self._cache = (th.copy(), self.spec.atmosphere(th))
        return self._cache[1]

    def forward(self, theta, stream=None):
        import torch
        atmo = self._atmo(theta)
        S = torch.empty(self.shape, dtype=torch.float64, device=self.g_psi.device)
        A = torch.empty_like(S)
        lst = C.byref(self._list) if self.use_list else None
        _check(lib().ckv_soft_forward(C.byref(self._segs), C.byref(self._showers), C.byref(self.params),
                                      atmo.handle, self.tels.handle, C.c_void_p(self.n_b.data_ptr()),
                                      C.c_void_p(S.data_ptr()), C.c_void_p(A.data_ptr()), lst,
                                      C.c_void_p(self.result_raw.data_ptr()),
                                      C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                      _stream_ptr(stream)))
        self._check_device("forward")
        if self.use_list:
            self._list_theta = np.array(theta, dtype=np.float64, copy=True)
        return S, A

    def _check_device(self, what: str):
        """Raises when the device reported bad shower offsets or an oversized tile
        (synchronises with the stream), until a clean pass of this kind proves the
        model free of both."""
        if self._clean[what]:
            return
        err = RunOutput(None, None, None, self.result_raw).result()["error"]
        if err:
            raise CkvError(f"soft {what}: device reported error flags {err} "
                           "(1: bad seg_offsets, 2: a 32-step tile with >= 2^30 frozen bunches)")
        self._clean[what] = self._bound_holds

    def backward_tables(self, theta, gS, gA, stream=None):
        """Device dL/dpsi (n_nodes) and dL/dP (5 x n_nodes)."""
        atmo = self._atmo(theta)
        gS = gS.to(self.g_psi.device, dtype=self.g_psi.dtype).contiguous()
        gA = gA.to(self.g_psi.device, dtype=self.g_psi.dtype).contiguous()
        # the list is valid for the theta of the forward that wrote it
        listed = self.use_list and self._list_theta is not None and \
            np.array_equal(self._list_theta, np.asarray(theta, dtype=np.float64))
        lst = C.byref(self._list) if listed else None
        _check(lib().ckv_soft_backward(C.byref(self._segs), C.byref(self._showers), C.byref(self.params),
                                       atmo.handle, self.tels.handle, C.c_void_p(self.n_b.data_ptr()),
                                       C.c_void_p(gS.data_ptr()), C.c_void_p(gA.data_ptr()),
                                       C.c_void_p(self.g_psi.data_ptr()), C.c_void_p(self.g_P.data_ptr()),
                                       lst, C.c_void_p(self.result_raw.data_ptr()),
                                       C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                       _stream_ptr(stream)))
        self._check_device("backward")
        return self.g_psi, self.g_P

    def grow_list(self) -> bool:
        """After a forward: enlarge the list if it was too small (synchronises);
        True when it was, so the next forward records a complete list."""
        if not self.use_list:
            return False
        n, cap = self.list_state()
        if 0 <= n <= cap:
            return False
        if n >= (1 << 62):
            self.use_list = False       # ids beyond the packed range: recompute everything
            return True
        self._alloc_list(int(n * 1.25) + 1024)
        return True

    def backward(self, theta, gS, gA, stream=None) -> np.ndarray:
        import torch
        g_psi, g_P = self.backward_tables(theta, gS, gA, stream)
        torch.cuda.synchronize()
        self.grow_list()
        g = self._g.cpu().numpy()
        n = g_psi.numel()
        return self.spec.backward(theta, self._atmo(theta), g[:n], g[n:])


def _soft_function():
    import torch

    class SoftResponse(torch.autograd.Function):
        """(S, A) = soft telescope response at atmosphere parameters theta.

        The backward pass runs the adjoint kernel (bunches recomputed from their
        random numbers) and the table chain rule in the library."""

        @staticmethod
        def forward(ctx, theta, model):
            ctx.model = model
            ctx.save_for_backward(theta)
            return model.forward(theta.detach().cpu().numpy())

        @staticmethod
        def backward(ctx, gS, gA):
            (theta,) = ctx.saved_tensors
            th = theta.detach().cpu().numpy()
            g = ctx.model.backward(th, gS, gA)
            return torch.as_tensor(g, dtype=theta.dtype, device=theta.device), None

    return SoftResponse


_SOFT = None


def soft_response(theta, model: SoftModel):
    """Differentiable (S, A) of shape (n_showers, n_tel) for torch tensor theta."""
    global _SOFT
    if _SOFT is None:
        _SOFT = _soft_function()
    return _SOFT.apply(theta, model)


# size of the static workspace of ckv_run_noalloc (CKV_NOALLOC_SCRATCH_MIB in include/ckv.h)
NOALLOC_SCRATCH_BYTES = 256 << 20
