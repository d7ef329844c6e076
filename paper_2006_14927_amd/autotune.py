"""Launch-shape autotuner for the bunch kernel.

Candidates are (steps per tile, waves per workgroup) pairs; each is timed on
the caller's own inputs with HIP events around whole ckv_run calls, and the
fastest is cached in a JSON file keyed by GPU architecture and a workload
signature (precision, step-count and shower-count magnitude, telescopes,
table nodes).  Every candidate computes the same records: the tile size and
wave count only change how work is distributed (tests check byte identity).
"""

from __future__ import annotations

import ctypes as C
import json
import math
import os
import statistics
from typing import Dict, List, Optional, Tuple

from . import ckv

DEFAULT_CANDIDATES: List[Tuple[int, int]] = [(ts, wv) for ts in (16, 32, 64) for wv in (16, 8, 4)]
CACHE_PATH = os.environ.get("CKV_AUTOTUNE_CACHE",
                            os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib",
                                         "autotune.json"))


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def signature(dsegs: "ckv.DeviceSegments", atmo: "ckv.Atmosphere", tels: "ckv.TelescopeArray",
              precision: int) -> str:
    from .build import source_hash
    n_nodes, _, _ = atmo.info()
    # the kernel sources are part of the key: a shape tuned on other kernels is not reused
    return (f"{_arch()}|src{source_hash()}|prec{precision}|seg2^{int(math.log2(max(dsegs.n, 1)))}"
            f"|show2^{int(math.log2(max(dsegs.n_showers, 1)))}|tel{tels.n}|nodes{n_nodes}")


def _load() -> Dict:
    try:
        with open(CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: Dict) -> None:
    os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
    tmp = f"{CACHE_PATH}.{os.getpid()}.tmp"      # one writer per file; replace is atomic
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE_PATH)


def cached(sig: str) -> Optional[Dict]:
    return _load().get(sig)


def _time_ms(runner: "ckv.Runner", reps: int) -> float:
    import torch
    hip = C.CDLL("libamdhip64.so")
    hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
    hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
    hip.hipEventSynchronize.argtypes = [C.c_void_p]
    hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
    hip.hipEventDestroy.argtypes = [C.c_void_p]
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    times = []
    for _ in range(reps):
        b, e = C.c_void_p(), C.c_void_p()
        hip.hipEventCreate(C.byref(b))
        hip.hipEventCreate(C.byref(e))
        hip.hipEventRecord(b, sp)
        runner.run(stream)
        hip.hipEventRecord(e, sp)
        hip.hipEventSynchronize(e)
        ms = C.c_float()
        hip.hipEventElapsedTime(C.byref(ms), b, e)
        times.append(ms.value)
        hip.hipEventDestroy(b)
        hip.hipEventDestroy(e)
    return statistics.median(times)


def tune(dsegs: "ckv.DeviceSegments", atmo: "ckv.Atmosphere", tels: "ckv.TelescopeArray",
         params: "ckv._Params", capacity: int, *, candidates=None, reps: int = 3,
         use_cache: bool = True) -> Dict:
    """Fastest (tile_segments, waves_per_group) for these inputs; cached."""
    import torch
    sig = signature(dsegs, atmo, tels, params.precision)
    if use_cache:
        hit = cached(sig)
        if hit is not None:
            return hit
    table = []
    for ts, wv in (candidates or DEFAULT_CANDIDATES):
        p = ckv._Params.from_buffer_copy(params)
        p.tile_segments, p.waves_per_group = ts, wv
        p.event_begin = p.event_end = None
        r = ckv.Runner(dsegs, atmo, tels, p, capacity, want_ids=False)
        r.run()
        torch.cuda.synchronize()
        res = r.run().result()
        torch.cuda.synchronize()
        if res["overflow"] or res["error"]:
            continue
        table.append({"tile_segments": ts, "waves_per_group": wv, "ms": _time_ms(r, reps)})
        del r
    if not table:
        raise ckv.CkvError("autotune: no candidate ran")
    best = min(table, key=lambda x: x["ms"])
    entry = {"tile_segments": best["tile_segments"], "waves_per_group": best["waves_per_group"],
             "ms": best["ms"], "table": table}
    if use_cache:
        cache = _load()
        cache[sig] = entry
        _store(cache)
    return entry


def apply(params: "ckv._Params", entry: Dict) -> "ckv._Params":
    p = ckv._Params.from_buffer_copy(params)
    p.tile_segments = int(entry["tile_segments"])
    p.waves_per_group = int(entry["waves_per_group"])
    return p
