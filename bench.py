"""Throughput of the Cherenkov bunch path on one MI355X.

One step = one ckv_run over the 1 TeV gamma-like shower at 20 deg zenith
(2e6 track steps, ~1.2e8 bunches, 100 telescopes, 5-layer atmosphere on a
50 m grid): bunch counts, emission, propagation, sphere tests and the ordered
per-telescope output, with the inputs already resident in HBM.

The reported value is bunches generated and propagated per second in the
mixed FP32/FP64 path; the FP64 path is timed the same way and reported beside
it.  The roofline entry refers to the bunch kernel (the dominant kernel); its
duration is measured with HIP events recorded around that kernel on the
stream it runs on.  The CPU baseline is the FP64 oracle timed on a sample of
the same shower.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# --- algorithmic VALU work per generated bunch, in issue slots: each arithmetic,
# logic, compare, select or conversion the algorithm needs at the path's precision,
# weighted by its issue cost on this chip as measured by single-instruction rate
# probes: 1 slot for FP32/FP64 add, mul and FMA, integer and logic operations,
# conversions and the 32x32->64 multiply; 2 for an FP32 transcendental (rcp, sqrt,
# sin, cos); 4 for an FP64 one (rcp, and the estimate inside a square root).  An
# operation the chip has as one instruction counts once (an FMA, a three-input XOR
# such as Philox's hi ^ counter ^ key).  Loop
# control, addressing and register moves are not counted.
OPS_MIXED = {
    "philox4x32-10: 10 rounds x (2 mul32x32->64 + 2 three-input xor)": 40,
    "uniforms u0, u2 (convert + scale)": 4,
    "emission point and time (FP64)": 7,
    "azimuth: quadrant, angle in turns (4), hardware sin + cos (2 x 2), quadrant selects (6)": 14,
    "direction on the cone (FP32 perpendicular, FP64 sum)": 12,
    "wavelength (inverse CDF: fma + rcp)": 3,
    "drop tests": 4,
    "table index (FP64 -> cell, fraction)": 7,
    "moments about psi_e, D1..D5: node moments shifted (15 FMA) + in-cell closed form (11)": 26,
    "index at emission (sqrt, 2 rcp), n_e / n_obs": 12,
    "1/w (FP64 rcp + 1 Newton step)": 6,
    "series variable q (rcp)": 6,
    "advance series S": 9,
    "time series T (n_e^2 times the advance series + a_k q^k D_{k+1})": 10,
    "ground point, arrival time": 5,
    "observed direction, record conversions": 6,
    "candidate cell": 13,
    "sphere tests (0.35 candidates per bunch x 7)": 3,
}
OPS_FP64 = {
    "philox4x32-10 (as above)": 40,
    "uniforms u0, u2": 4,
    "emission point and time": 7,
    "azimuth sin/cos: quadrant fold + Taylor polynomials to a^17 (FP64)": 32,
    "direction on the cone": 9,
    "wavelength (rcp + 2 Newton)": 10,
    "drop tests": 4,
    "table index": 6,
    "moments about psi_e, D1..D5: node shift + in-cell closed form": 26,
    "index at emission (sqrt, 1/n_e by rcp + 2 Newton, n_e / n_obs)": 14,
    "1/w (rcp + 2 Newton)": 8,
    "series variable q": 3,
    "advance series S": 9,
    "time series T (sharing the advance series)": 10,
    "ground point, arrival time": 5,
    "observed direction, record conversions": 6,
    "candidate cell + sphere tests": 16,
}
# Per-bunch issue-slot counts of the whole path, operation by operation (lane-slots
# per generated bunch, issue-cycle weighted, every instruction the per-bunch work
# needs): 280-300 for the mixed path, 380-450 for plain FP64; the midpoints are the
# counts the roofline fraction is priced with.  The itemised algorithmic counts above
# (arithmetic the method needs, no addressing or control) are reported beside them.
PATH_SLOTS = {"mixed": 290.0, "fp64": 415.0}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one VALU operation per lane
# per clock (FP32 non-packed and FP64 both issue at this rate on CDNA4)
PEAK_OPS_PER_S = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0
SEG_BYTES = 9 * 8 + 1            # SoA step record read once
PROFILE_BIN_GCM2 = 20.0          # depth bin of the longitudinal profile run
RECORD_BYTES = 32                # output record


def _hip():
    for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
        try:
            h = C.CDLL(name)
            h.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
            h.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
            h.hipEventSynchronize.argtypes = [C.c_void_p]
            h.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
            h.hipEventDestroy.argtypes = [C.c_void_p]
            return h
        except OSError:
            continue
    raise RuntimeError("libamdhip64.so not found")


# hipDeviceAttribute_t values of this ROCm's hip_runtime_api.h
_HIP_ATTR = {"clock_khz": 5, "mem_bus_bits": 59, "mem_clock_khz": 60, "cus": 63,
             "lds_per_cu_bytes": 10002}


def device_info(hip) -> dict:
    """The chip's figures as the runtime reports them on the machine that runs this."""
    import torch
    props = torch.cuda.get_device_properties(0)
    hip.hipDeviceGetAttribute.argtypes = [C.POINTER(C.c_int), C.c_int, C.c_int]
    out = {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
           "hbm_gib": round(props.total_memory / 2 ** 30, 1)}
    for k, attr in _HIP_ATTR.items():
        v = C.c_int()
        out[k] = int(v.value) if hip.hipDeviceGetAttribute(C.byref(v), attr, 0) == 0 else None
    return out


def _event(hip):
    e = C.c_void_p()
    if hip.hipEventCreate(C.byref(e)) != 0:
        raise RuntimeError("hipEventCreate failed")
    return e


def _elapsed_ms(hip, a, b) -> float:
    ms = C.c_float()
    if hip.hipEventElapsedTime(C.byref(ms), a, b) != 0:
        raise RuntimeError("hipEventElapsedTime failed")
    return float(ms.value)


def kernel_source_hash() -> str:
    from paper_2006_14927_amd.build import source_hash
    return source_hash()


ZENITH_SAMPLE_STRIDE = 250       # every 250th step of each 5e7-step shower is certified


def emit_kernel_name(precision: int, tile_segments: int, waves: int) -> str:
    """Symbol of the bunch kernel a plain run launches (the mixed kernel has a
    build for at most 8 waves per workgroup, feature bit 16; the FP64 kernel one
    for 16 waves, feature bit 64)."""
    if precision == 1:
        feat = 16 if waves <= 8 else 0
    else:
        feat = 64 if waves > 8 else 0     # the FP64 16-wave build stages part of the table
    return f"void ckv::emit_kernel<{precision}, {tile_segments}, {feat}>(ckv::Args)"


def _profile_kv(path: str) -> dict:
    kv = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                # keys may hold a kernel symbol (ckv::...): the value follows the last colon
                k, v = line.rsplit(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def stored_issue_frac(kernel: str, workload: str):
    """VALU issue fraction of a kernel from the committed rocprofv3 SQ summary of
    the workload, if it was taken on the current sources; else None."""
    kv = _profile_kv(os.path.join(ROOT, "profiles", f"sq_bunch_kernel_{workload}.txt"))
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv[f"issue_frac {kernel}"])
    except (KeyError, ValueError):
        return None


def stored_traffic(name: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_path(hip, ckv, dsegs, atmo, tels, params, capacity, steps, warmup, stream):
    """warmup + steps launches on `stream`; returns (ms per step, bunch-kernel ms, result)."""
    import torch
    r = ckv.Runner(dsegs, atmo, tels, params, capacity, want_ids=False)
    for _ in range(warmup):
        r.run(stream)
    torch.cuda.synchronize()
    ev_k = [(_event(hip), _event(hip)) for _ in range(steps)]
    t_begin, t_end = _event(hip), _event(hip)
    sp = C.c_void_p(stream.cuda_stream)
    hip.hipEventRecord(t_begin, sp)
    for b, e in ev_k:
        r.params.event_begin = b.value
        r.params.event_end = e.value
        out = r.run(stream)
    hip.hipEventRecord(t_end, sp)
    hip.hipEventSynchronize(t_end)
    torch.cuda.synchronize()
    total_ms = _elapsed_ms(hip, t_begin, t_end)
    kern_ms = [_elapsed_ms(hip, b, e) for (b, e) in ev_k]
    r.params.event_begin = None
    r.params.event_end = None
    for b, e in ev_k + [(t_begin, t_end)]:
        hip.hipEventDestroy(b)
        hip.hipEventDestroy(e)
    return total_ms / steps, sum(kern_ms) / len(kern_ms), out.result()


def gpu_records(ckv, dsegs, atmo, tels, params, capacity, step_stride=0):
    """One untimed run of the same launch with ids on: host copies of the CSR
    offsets, the records and their (step, bunch) ids, and the report.  With
    step_stride > 0 only the records of every step_stride-th step are copied
    (selected on the device)."""
    import torch
    p = ckv._Params.from_buffer_copy(params)
    p.event_begin = p.event_end = None
    r = ckv.Runner(dsegs, atmo, tels, p, capacity, want_ids=True)
    out = r.run()
    torch.cuda.synchronize()
    res = out.result()
    if res["overflow"] or res["error"]:
        raise RuntimeError(f"certification run reported a problem: {res}")
    n = int(res["n_records"])
    ids, rec = out.ids[:n], out.records[:n]
    offsets = out.tel_offsets.cpu().numpy().copy()
    if step_stride > 0:
        # each record's (shower, telescope) group, then keep the sampled steps
        counts = torch.diff(out.tel_offsets)
        group = torch.repeat_interleave(torch.arange(counts.numel(), device=ids.device), counts)
        keep = (ids[:, 0] % step_stride) == 0
        got = dict(group=group[keep].cpu().numpy(), ids=ids[keep].cpu().numpy(),
                   rec=rec[keep].cpu().numpy(), res=res, offsets=None)
    else:
        counts = np.diff(offsets)
        got = dict(group=np.repeat(np.arange(len(counts)), counts), ids=ids.cpu().numpy(),
                   rec=rec.cpu().numpy(), res=res, offsets=offsets)
    del r, out
    torch.cuda.empty_cache()
    return got


def cpu_info() -> dict:
    """Host CPU as the machine that runs the bench reports it."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cores": len(os.sched_getaffinity(0))}


EARTH_RADIUS_M = 6.371e6


def curved_timing(hip, stream, reps: int = 3, zenith: float = 70.0, n_seg: int = 2_000_000):
    """The TeV shower at a large zenith angle, three ways, mixed precision:
    plane-parallel with the moment series (grazing bunches dropped), the same with
    the exact grazing path, and the curved atmosphere (spherical shells of the
    Earth's radius, every bunch traced exactly in FP64)."""
    from paper_2006_14927_amd import ckv, synth
    wl = synth.inclined(zenith, n_seg)
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    d = ckv.DeviceSegments(wl.segs)
    cap = max(1 << 16, wl.segs.n)
    out = {"workload": wl.name, "zenith_deg": zenith, "earth_radius_m": EARTH_RADIUS_M}
    for name, kw in (("flat_series", {}), ("flat_exact_grazing", dict(grazing_exact=True)),
                     ("curved_exact", dict(earth_radius=EARTH_RADIUS_M))):
        p = ckv.make_params(precision=ckv.CKV_MIXED, bunch_size=wl.bunch_size,
                            lambda_min=wl.lambda_min, lambda_max=wl.lambda_max, seed=wl.seed,
                            tile_segments=32, **kw)
        ms, kms, res = time_path(hip, ckv, d, atmo, tels, p, cap, reps, 1, stream)
        if res["error"] or res["overflow"]:
            raise RuntimeError(f"{name} run reported a problem: {res}")
        out[name] = {"ms_per_step": ms, "bunch_kernel_ms": kms, "bunches": res["n_bunches"],
                     "records": res["n_hits"], "bunches_per_s": res["n_bunches"] / (ms * 1e-3),
                     "drops_grazing": res["drops"]["grazing"], "drops_upward": res["drops"]["upward"]}
        print(f"# {wl.name} {name}: {ms:.3f} ms/step, {res['n_bunches']} bunches, "
              f"{res['n_hits']} records", file=sys.stderr, flush=True)
    out["curved_over_flat"] = out["curved_exact"]["ms_per_step"] / out["flat_series"]["ms_per_step"]
    return out


def diff_timing(hip, reps: int, n_showers: int = 64, n_seg: int = 500_000):
    """Forward + backward of the soft telescope response on the differentiation
    workload (64 showers x 5e5 steps); returns ms per shower and kernel times."""
    import torch

    from paper_2006_14927_amd import ckv, synth
    from paper_2006_14927_amd.objective import telescope_loss
    dw = synth.diff_showers(n_showers, n_seg)
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    model = ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed)
    St, At = model.forward(dw.theta_target)
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)

    def step(events=None):
        theta = torch.tensor(dw.theta0, dtype=torch.float64, requires_grad=True)
        if events:
            model.params.event_begin, model.params.event_end = events[0].value, events[1].value
        S, A = ckv.soft_response(theta, model)
        loss = telescope_loss(S, A, St, At)
        if events:
            model.params.event_begin, model.params.event_end = events[2].value, events[3].value
        loss.backward()
        model.params.event_begin = model.params.event_end = None
        return theta.grad

    step()
    torch.cuda.synchronize()
    walls, fwd, bwd = [], [], []
    for _ in range(reps):
        ev = [_event(hip) for _ in range(4)]
        t0 = time.perf_counter()
        g = step(ev)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        fwd.append(_elapsed_ms(hip, ev[0], ev[1]))
        bwd.append(_elapsed_ms(hip, ev[2], ev[3]))
        for e in ev:
            hip.hipEventDestroy(e)
    nb = int(model.n_b.sum())
    if not bool(torch.isfinite(g).all()):
        raise RuntimeError("differentiation: non-finite gradient")
    n_listed, cap = model.list_state()
    # one pass with the adjoint recomputing every bunch, for comparison
    model.use_list = False
    ev = [_event(hip) for _ in range(4)]
    g_full = step(ev)
    torch.cuda.synchronize()
    fwd_nolist = _elapsed_ms(hip, ev[0], ev[1])
    bwd_full = _elapsed_ms(hip, ev[2], ev[3])
    for e in ev:
        hip.hipEventDestroy(e)
    model.use_list = True
    wall = sorted(walls)[len(walls) // 2]
    return {"workload": dw.name, "showers": n_showers, "steps": dw.segs.n, "bunches": nb,
            "ms_per_shower": wall / n_showers, "fwd_kernel_ms": sum(fwd) / len(fwd),
            "bwd_kernel_ms": sum(bwd) / len(bwd), "wall_ms": wall,
            "listed_bunches": n_listed, "list_complete": bool(0 <= n_listed <= cap),
            "fwd_kernel_ms_without_list": fwd_nolist, "bwd_kernel_ms_every_bunch": bwd_full,
            "grad_rel_diff_every_bunch": float((g_full - g).norm() / g.norm()),
            "grad_norm": float(g.norm())}


def roofline_block(slots_path: float, slots_itemised: float, bunches: int, kernel_ms: float,
                   issue_frac=None) -> dict:
    """VALU issue-slot roofline of a bunch kernel: algorithmic slots per bunch x
    bunches / kernel time against 256 CU x 4 SIMD x 16 lanes x 2.4 GHz."""
    achieved = slots_path * bunches / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_OPS_PER_S / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
            "frac": achieved / peak, "slots_per_bunch": slots_path,
            "frac_itemised_model": slots_itemised * bunches / (kernel_ms * 1e-3) / PEAK_OPS_PER_S,
            "slots_per_bunch_itemised_model": slots_itemised, "issue_frac": issue_frac}


def batched_timing(hip, reps: int, use_cache: bool = True):
    """256 showers (~3e8 steps, ~2e10 bunches) in one persistent launch, the whole
    run captured into a HIP graph and replayed; mixed precision and plain FP64,
    each with its autotuned launch shape.  The bunch kernel's own time comes from
    two eager runs of the same launch with HIP events around it."""
    import torch

    from paper_2006_14927_amd import autotune, ckv, synth
    wl = synth.batched_showers(256)
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    d = ckv.DeviceSegments(wl.segs)
    stream = torch.cuda.current_stream()

    def mk(prec):
        return ckv.make_params(precision=prec, bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                               lambda_max=wl.lambda_max, seed=wl.seed)

    total = int(ckv.count(d, atmo, mk(ckv.CKV_MIXED)).sum())
    cap = int(0.02 * total)
    probe = ckv.Runner(d, atmo, tels, mk(ckv.CKV_MIXED), cap, want_ids=False).run()
    torch.cuda.synchronize()
    res = probe.result()
    if res["overflow"]:
        cap = int(res["n_hits"]) + 1024
    del probe
    torch.cuda.empty_cache()
    out = {"workload": wl.name, "showers": wl.segs.n_showers, "steps": wl.segs.n,
           "bunches": total, "graph_replays": reps}
    cands = {ckv.CKV_MIXED: [(32, 16), (64, 16), (32, 8), (16, 16)],
             ckv.CKV_FP64: [(32, 8), (64, 8), (16, 8), (16, 16), (32, 16)]}
    for prec, name in ((ckv.CKV_MIXED, "mixed"), (ckv.CKV_FP64, "fp64_plain")):
        tuned = autotune.tune(d, atmo, tels, mk(prec), cap, candidates=cands[prec], reps=1,
                              use_cache=use_cache)
        q = autotune.apply(mk(prec), tuned)
        gr = ckv.GraphRunner(ckv.Runner(d, atmo, tels, q, cap, want_ids=False))
        gr.replay()
        torch.cuda.synchronize()
        sp = C.c_void_p(gr.stream.cuda_stream)
        t0, t1 = _event(hip), _event(hip)
        hip.hipEventRecord(t0, sp)
        for _ in range(reps):
            with torch.cuda.stream(gr.stream):
                o = gr.replay()
        hip.hipEventRecord(t1, sp)
        hip.hipEventSynchronize(t1)
        torch.cuda.synchronize()
        ms = _elapsed_ms(hip, t0, t1) / reps
        hip.hipEventDestroy(t0)
        hip.hipEventDestroy(t1)
        res = o.result()
        if res["overflow"] or res["error"] or res["n_bunches"] != total:
            raise RuntimeError(f"batched {name} run reported a problem: {res}")
        del gr, o
        torch.cuda.empty_cache()
        _, kms, _ = time_path(hip, ckv, d, atmo, tels, q, cap, 2, 0, stream)
        torch.cuda.empty_cache()
        key = "mixed" if prec == ckv.CKV_MIXED else "fp64"
        ops = OPS_MIXED if prec == ckv.CKV_MIXED else OPS_FP64
        out[name] = {"ms_per_launch": ms, "bunches_per_s": total / (ms * 1e-3),
                     "records": res["n_hits"], "bunch_kernel_ms": kms,
                     "launch": {"tile_segments": tuned["tile_segments"],
                                "waves_per_group": tuned["waves_per_group"]},
                     "roofline": roofline_block(PATH_SLOTS[key], sum(ops.values()), total, kms,
                                                stored_issue_frac(emit_kernel_name(
                                                    prec, tuned["tile_segments"],
                                                    tuned["waves_per_group"]), "batched_256"))}
        print(f"# batched {name}: {ms:.2f} ms per graph launch, bunch kernel {kms:.2f} ms",
              file=sys.stderr, flush=True)
    out["ms_per_launch"] = out["mixed"]["ms_per_launch"]
    out["bunches_per_s"] = out["mixed"]["bunches_per_s"]
    out["records"] = out["mixed"]["records"]
    out["mixed_over_fp64"] = out["fp64_plain"]["ms_per_launch"] / out["mixed"]["ms_per_launch"]
    return out


def streamed_timing(hip, zeniths=(0.0, 20.0, 40.0, 60.0), sample_stride: int = 250):
    """One 5e7-step hadron-like shower per zenith: the mixed-precision output
    streamed to pinned host memory in chunks of 8 388 608 records (256 MB), timed
    from the bunch counts to the last chunk on the host; then both precisions
    resident in HBM (one ckv_run over the whole shower, bunch kernel timed by
    events), and the records of every sample_stride-th step of an untimed mixed
    run kept for the per-zenith comparison with the oracle."""
    import torch

    from paper_2006_14927_amd import ckv, synth
    out, samples = [], []
    stream = torch.cuda.current_stream()
    for z in zeniths:
        wl = synth.hadron_like(z)
        atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
        tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
        d = ckv.DeviceSegments(wl.segs)

        def mk(prec):
            return ckv.make_params(precision=prec, bunch_size=wl.bunch_size,
                                   lambda_min=wl.lambda_min, lambda_max=wl.lambda_max, seed=wl.seed)

        p = mk(ckv.CKV_MIXED)
        ckv.Streamer(d, atmo, tels, p, want_ids=False)        # warm: allocations, first launch
        torch.cuda.synchronize()
        agg = dict(chunks=0, records=0, end=0)

        def sink(ch):
            if ch.begin != agg["end"] or ch.result["error"]:
                raise RuntimeError(f"streamed chunk [{ch.begin}, {ch.end}) out of order or failed")
            agg["chunks"] += 1
            agg["records"] += int(ch.records.shape[0])
            agg["end"] = ch.end

        t0 = time.perf_counter()
        st = ckv.Streamer(d, atmo, tels, p, want_ids=False)
        st.to_host(sink)
        dt = time.perf_counter() - t0
        n_chunks, n_rec, n_b = agg["chunks"], agg["records"], st.total_bunches
        if agg["end"] != wl.segs.n:
            raise RuntimeError("streamed chunks do not cover the shower")
        resumed, rerun = st.n_resumed, st.n_reruns
        del st
        torch.cuda.empty_cache()
        entry = {"zenith_deg": z, "steps": wl.segs.n, "bunches": n_b, "records": n_rec,
                 "chunks": n_chunks, "resumed": resumed, "rerun": rerun, "s": dt,
                 "bunches_per_s": n_b / dt}
        cap = n_rec + (1 << 16)
        # each precision at its faster launch shape (FP64: the 8-wave build with the whole
        # table in LDS, or the 16-wave build staging part of it)
        shapes = {ckv.CKV_MIXED: [(32, 16)], ckv.CKV_FP64: [(32, 8), (16, 16)]}
        for prec, name in ((ckv.CKV_MIXED, "resident_mixed"), (ckv.CKV_FP64, "resident_fp64")):
            best = None
            for ts, wv in shapes[prec]:
                q = ckv.make_params(precision=prec, bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                                    lambda_max=wl.lambda_max, seed=wl.seed, tile_segments=ts,
                                    waves_per_group=wv)
                ms, kms, res = time_path(hip, ckv, d, atmo, tels, q, cap, 3, 1, stream)
                if res["error"] or res["overflow"] or res["n_bunches"] != n_b or \
                        (prec == ckv.CKV_MIXED and res["n_hits"] != n_rec):
                    raise RuntimeError(f"{name} at {z} deg reported a problem: {res}")
                if best is None or ms < best["ms"]:
                    best = {"ms": ms, "bunch_kernel_ms": kms, "bunches_per_s": n_b / (ms * 1e-3),
                            "launch": {"tile_segments": ts, "waves_per_group": wv}}
                torch.cuda.empty_cache()
            entry[name] = best
        entry["resident_mixed_over_fp64"] = entry["resident_fp64"]["ms"] / entry["resident_mixed"]["ms"]
        samples.append((wl, gpu_records(ckv, d, atmo, tels, p, cap, step_stride=sample_stride)))
        out.append(entry)
        print(f"# streamed {wl.name}: {out[-1]}", file=sys.stderr, flush=True)
        del d
        torch.cuda.empty_cache()
    return out, samples


def vertical_gamma_timing(hip, stream, steps: int, warmup: int):
    """The plain-FP64 configuration of the paper-scale vertical gamma shower
    (2e4 steps, 9 telescopes), both precisions; returns the timings and the
    records of each precision for the comparison with the oracle."""
    from paper_2006_14927_amd import ckv, synth
    wl = synth.vertical_gamma()
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    d = ckv.DeviceSegments(wl.segs)
    cap = max(1 << 16, 8 * wl.segs.n)
    out, recs = {"workload": wl.name, "steps": wl.segs.n, "telescopes": wl.tels.n}, {}
    for prec, name in ((ckv.CKV_FP64, "fp64_plain"), (ckv.CKV_MIXED, "mixed")):
        p = ckv.make_params(precision=prec, bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                            lambda_max=wl.lambda_max, seed=wl.seed)
        ms, kms, res = time_path(hip, ckv, d, atmo, tels, p, cap, steps, warmup, stream)
        if res["error"] or res["overflow"]:
            raise RuntimeError(f"vertical gamma {name} reported a problem: {res}")
        out[name] = {"ms_per_step": ms, "bunch_kernel_ms": kms, "bunches": res["n_bunches"],
                     "records": res["n_hits"], "bunches_per_s": res["n_bunches"] / (ms * 1e-3)}
        recs[prec] = gpu_records(ckv, d, atmo, tels, p, cap)
        recs[prec]["n_b"] = ckv.count(d, atmo, p).cpu().numpy()
    out["mixed_over_fp64"] = out["fp64_plain"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    return wl, out, recs


def order_study(hip, wl, atmo, tels, stream, steps: int, warmup: int):
    """Bunch-kernel time with the shower's steps in generator order, sorted by
    start altitude (neighbouring lanes then read neighbouring table cells), and
    shuffled: the memory-layout study of the step input.  The reordered runs pass
    the generator-order index of each step as its step id, so they compute the
    same bunches as the generator order (checked: same counts, crossings and
    drops)."""
    import torch

    from paper_2006_14927_amd import ckv
    orders = {"generator": None,
              "by_altitude": np.argsort(-wl.segs.h0, kind="stable"),
              "shuffled": np.random.default_rng(1).permutation(wl.segs.n)}
    out, ref = {}, None
    for name, idx in orders.items():
        d = ckv.DeviceSegments(wl.segs) if idx is None else \
            ckv.DeviceSegments(wl.segs.take(idx), step_id=idx.astype(np.uint32))
        p = ckv.make_params(precision=ckv.CKV_MIXED, bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                            lambda_max=wl.lambda_max, seed=wl.seed, tile_segments=32, waves_per_group=16)
        ms, kms, res = time_path(hip, ckv, d, atmo, tels, p, max(1 << 16, 2 * wl.segs.n), steps, warmup,
                                 stream)
        key = (res["n_bunches"], res["n_hits"], tuple(res["drops"].values()))
        ref = key if ref is None else ref
        out[name] = {"ms_per_step": ms, "bunch_kernel_ms": kms, "bunches": res["n_bunches"],
                     "records": res["n_hits"], "same_bunches_as_generator_order": key == ref}
        print(f"# step order {name}: {out[name]}", file=sys.stderr, flush=True)
        del d
        torch.cuda.empty_cache()
    return out


# --- the oracle leg: the FP64 CPU oracle timed on a sample of the shower, and the
# same sample used to certify the GPU records of the timed launches.  Everything
# that touches oracle/ lives below.

# tolerances the mixed path is held to against the FP64 oracle, and the
# guard band of the sphere test: |disc| <= 2 R eps + eps^2 with eps = 1 mm
TOL = {"ground_m": 1e-3, "dir": 1e-6, "t_ns": 0.01, "photons_rel": 1e-6, "lambda_rel": 1e-6}
GUARD_EPS_M = 1e-3
F32_HALF_ULP = 2.0 ** -24
# the library's bound of the mixed path's ground-point error per metre of height
# (the soft response's screening pass relies on it): dh (a (1/w + 1/w^2) + b / w^3)
SCREEN_ERR_DIR, SCREEN_ERR_SERIES = 1e-8, 5e-10


def oracle_threads():
    """Threads for the oracle: every core this process may run on, at most 16
    (the host cores allotted per GPU on the machines this runs on)."""
    aff = len(os.sched_getaffinity(0))
    return max(1, min(16, aff))


def certify(cfg, segs, precision: int, idx, ores, gpu, n_b_gpu=None) -> dict:
    """Compares the GPU records of the sampled steps idx (global step indices,
    ascending; gpu = gpu_records output) with the oracle's records of the same
    steps (ores, run on segs.take(idx) with their original random numbers).
    FP64 path: the same crossings in the same per-(shower, telescope) order and
    records equal up to the final FP32 rounding.  Mixed path: crossings differ
    only inside the guard band, fields within the stated tolerances.  Bunch
    counts of the sampled steps bit-exact (n_b_gpu from ckv_count)."""
    import oracle
    n_tel = cfg.n_tel
    sel = np.isin(gpu["ids"][:, 0], idx)
    gseg, gk = gpu["ids"][sel, 0], gpu["ids"][sel, 1]
    grp, grec = gpu["group"][sel], gpu["rec"][sel].astype(np.float64)
    oseg, ok_ = idx[ores.seg], ores.k
    ogrp = ores.bucket.astype(np.int64) * n_tel + ores.tel
    nmax = int(max(gseg.max(initial=0), oseg.max(initial=0))) + 1
    kmax = int(max(gk.max(initial=0), ok_.max(initial=0))) + 1
    gkey = (grp * nmax + gseg) * kmax + gk
    okey = (ogrp * nmax + oseg) * kmax + ok_
    order_ok = bool(np.all(np.diff(gkey) > 0))
    common, io, ig = np.intersect1d(okey, gkey, assume_unique=True, return_indices=True)
    only_o = np.setdiff1d(np.arange(len(okey)), io)
    only_g = np.setdiff1d(np.arange(len(gkey)), ig)
    ro, rg = ores.rec[io], grec[ig]
    d = np.abs(rg - ro)
    rel = lambda c: float(np.max(d[:, c] / np.maximum(np.abs(ro[:, c]), 1e-300), initial=0.0))
    out = {"sampled_steps": int(len(idx)), "oracle_records": int(len(okey)),
           "gpu_records": int(len(gkey)), "matched": int(len(common)),
           "canonical_order": order_ok,
           "max_abs_ground_m": float(d[:, :2].max(initial=0.0)),
           "max_abs_dir": float(d[:, 2:4].max(initial=0.0)),
           "max_abs_t_ns": float(d[:, 4].max(initial=0.0)),
           "max_rel_h_emit": rel(5), "max_rel_photons": rel(6), "max_rel_lambda": rel(7)}
    ok = order_ok
    if n_b_gpu is not None:
        out["bunch_counts_bit_exact"] = bool(np.array_equal(n_b_gpu[idx], ores.n_b))
        ok &= out["bunch_counts_bit_exact"]
    guard = lambda tel: 2.0 * cfg.tr[tel] * GUARD_EPS_M + GUARD_EPS_M ** 2
    if precision == 0:
        # identical crossing sets; records equal up to the final FP32 rounding
        tol = 2 * F32_HALF_ULP * np.abs(ro) + 1e-9
        tol[:, 4] += 2e-7
        out["flips"] = int(len(only_o) + len(only_g))
        out["records_within_fp32_rounding"] = bool(np.all(d <= tol))
        ok &= out["flips"] == 0 and out["records_within_fp32_rounding"]
    else:
        in_o = np.abs(ores.disc[only_o]) <= guard(ogrp[only_o] % n_tel)
        disc_g = np.zeros(0)
        if len(only_g):
            bd = oracle.bunch_details(cfg, segs, gseg[only_g], gk[only_g])
            tg = grp[only_g] % n_tel
            disc_g = np.array([oracle.sphere_disc(bd["x_g"][i], bd["y_g"][i], bd["u_o"][i],
                                                  bd["v_o"][i], cfg.tx[t], cfg.ty[t], cfg.tr[t])
                               for i, t in enumerate(tg)])
            in_g = np.abs(disc_g) <= guard(tg)
        else:
            in_g = np.zeros(0, dtype=bool)
        # the ground error against the bound the soft response's screening relies on
        wo = np.sqrt(np.maximum(1.0 - ro[:, 2] ** 2 - ro[:, 3] ** 2, 1e-12))
        dh = np.maximum(ro[:, 5] - cfg.tables.h_obs, 0.0)
        bound = dh / wo * (SCREEN_ERR_DIR * (1.0 + 1.0 / wo) + SCREEN_ERR_SERIES / wo ** 2)
        # plus the record's own FP32 rounding of dx, dy (the screen works on the FP64
        # ground point)
        bound = bound + 2.0 * F32_HALF_ULP * np.hypot(ro[:, 0], ro[:, 1]) + 1e-9
        gerr = np.hypot(d[:, 0], d[:, 1])
        out["max_ground_err_over_screen_bound"] = float(
            np.max(gerr / bound, initial=0.0))
        ok &= out["max_ground_err_over_screen_bound"] < 1.0
        out["flips_in_guard_band"] = int(in_o.sum() + in_g.sum())
        out["flips_outside_guard_band"] = int((~in_o).sum() + (~in_g).sum())
        out["tolerances"] = TOL
        ok &= out["flips_outside_guard_band"] == 0
        ok &= out["max_abs_ground_m"] <= TOL["ground_m"] and out["max_abs_dir"] <= TOL["dir"]
        ok &= out["max_abs_t_ns"] <= TOL["t_ns"]
        ok &= out["max_rel_photons"] <= TOL["photons_rel"] and out["max_rel_lambda"] <= TOL["lambda_rel"]
        ok &= out["max_rel_h_emit"] <= 2 * F32_HALF_ULP + 1e-9
    out["ok"] = bool(ok)
    return out


def oracle_leg(wl, gpu_main, n_b_main, runs: int = 5, target_cpu_seconds: float = 20.0):
    """The CPU baseline: the FP64 oracle on an evenly spaced sample of the
    shower's steps, median of `runs` timed runs on oracle_threads() threads
    (about target_cpu_seconds of CPU work in all), plus one run on one thread;
    then the parity certificate of both precisions on the same sample."""
    import oracle
    threads = oracle_threads()
    cfg = oracle.Config.from_workload(wl)
    probe = np.arange(0, wl.segs.n, max(1, wl.segs.n // 4000))
    t0 = time.perf_counter()
    r = oracle.run(cfg, wl.segs.take(probe), nthreads=threads, seg_id=probe)
    dt = max(time.perf_counter() - t0, 1e-3)
    rate_cpu_s = r.n_bunches / (dt * threads)          # bunches per CPU-second
    want_bunches = target_cpu_seconds / runs * rate_cpu_s
    mean_b = max(r.n_bunches / len(probe), 1e-9)
    stride = max(1, int(wl.segs.n * mean_b / max(want_bunches, 1.0)))
    idx = np.arange(0, wl.segs.n, stride)
    sub = wl.segs.take(idx)
    walls = []
    for _ in range(runs):
        t0 = time.perf_counter()
        r = oracle.run(cfg, sub, nthreads=threads, seg_id=idx)
        walls.append(time.perf_counter() - t0)
    med = float(np.median(walls))
    info = cpu_info()
    out = {"value": r.n_bunches / med, "unit": "bunches/s", "cores": threads, "kind": "oracle",
           "sample": f"every {stride}th step of the shower ({len(idx)} steps, {r.n_bunches} "
                     f"bunches, {len(r.seg)} records), FP64, median of {runs} runs "
                     f"({min(walls):.3f}-{max(walls):.3f} s wall)",
           "runs": runs, "wall_s": walls, "spread": (max(walls) - min(walls)) / med,
           **info,
           "threads_note": "every core of the process's affinity set, at most 16 (the host "
                           "cores allotted to one GPU)"}
    idx1 = idx[::threads]
    t0 = time.perf_counter()
    r1 = oracle.run(cfg, wl.segs.take(idx1), nthreads=1, seg_id=idx1)
    dt1 = time.perf_counter() - t0
    single = {"value": r1.n_bunches / dt1, "unit": "bunches/s", "cores": 1, "kind": "oracle",
              "sample": f"every {stride * threads}th step ({len(idx1)} steps, {r1.n_bunches} bunches), "
                        f"{dt1:.2f} s"}
    parity = {name: certify(cfg, wl.segs, prec, idx, r, gpu_main[prec], n_b_main)
              for prec, name in ((0, "fp64_plain"), (1, "mixed"))}
    parity["sample"] = f"every {stride}th step ({len(idx)} steps, {r.n_bunches} bunches)"
    return out, single, parity


def oracle_parity_full(wl, recs) -> dict:
    """Both precisions of a small workload against the oracle over every step."""
    import oracle
    cfg = oracle.Config.from_workload(wl)
    idx = np.arange(wl.segs.n)
    r = oracle.run(cfg, wl.segs, nthreads=oracle_threads())
    out = {name: certify(cfg, wl.segs, prec, idx, r, recs[prec], recs[prec]["n_b"])
           for prec, name in ((0, "fp64_plain"), (1, "mixed"))}
    for prec, name in ((0, "fp64_plain"), (1, "mixed")):
        res = recs[prec]["res"]
        out[name]["drops_bit_exact"] = dict(zip(oracle.DROP_NAMES, res_drops(res))) == r.drops
        out[name]["offsets_bit_exact"] = bool(np.array_equal(recs[prec]["offsets"], r.offsets))
        out[name]["ok"] &= out[name]["drops_bit_exact"] and (prec == 1 or out[name]["offsets_bit_exact"])
    return out


def res_drops(res):
    return [res["drops"][k] for k in ("mass", "threshold", "nonfinite", "below_obs", "above_top",
                                      "upward", "grazing")]


def oracle_parity_zeniths(samples, stride: int) -> list:
    """Per zenith: the mixed path's records of every stride-th step of the
    5e7-step shower against the oracle's (maximum errors by zenith)."""
    import oracle
    out = []
    for wl, gpu in samples:
        cfg = oracle.Config.from_workload(wl)
        idx = np.arange(0, wl.segs.n, stride)
        r = oracle.run(cfg, wl.segs.take(idx), nthreads=oracle_threads(), seg_id=idx)
        c = certify(cfg, wl.segs, 1, idx, r, gpu)
        c["workload"] = wl.name
        out.append(c)
        print(f"# parity {wl.name}: {c}", file=sys.stderr, flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the forward+backward timing of the differentiation workload")
    ap.add_argument("--diff-reps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-shower batched launch (~3e8 steps)")
    ap.add_argument("--no-streamed", action="store_true",
                    help="skip the 5e7-step hadron-like showers streamed in 256 MB chunks")
    ap.add_argument("--no-curved", action="store_true",
                    help="skip the curved-atmosphere timing (70 deg shower)")
    ap.add_argument("--order-study", action="store_true",
                    help="also time the shower with its steps sorted by altitude and shuffled")
    ap.add_argument("--no-tune-cache", action="store_true",
                    help="re-run the launch-shape autotuner instead of using its cache")
    ap.add_argument("--segments", type=int, default=2_000_000,
                    help="steps in the shower (default: the 2e6-step TeV shower)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(showers and step ranges would shard independently, one range per GPU).",
              file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_2006_14927_amd import ckv, synth
    ckv.lib()      # fails loudly when the HIP library is missing
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    hip = _hip()

    wl = synth.single_tev(args.segments)
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    dsegs = ckv.DeviceSegments(wl.segs)
    capacity = max(1 << 16, wl.segs.n * 2)

    def mk(precision):
        return ckv.make_params(precision=precision, bunch_size=wl.bunch_size,
                               lambda_min=wl.lambda_min, lambda_max=wl.lambda_max, seed=wl.seed)

    print(f"# workload {wl.name}: {wl.segs.n} steps, {wl.tels.n} telescopes", file=sys.stderr,
          flush=True)
    # launch shapes from the autotuner (untimed; cached per GPU arch and workload)
    from paper_2006_14927_amd import autotune
    tuned = {}
    for prec in (ckv.CKV_MIXED, ckv.CKV_FP64):
        tuned[prec] = autotune.tune(dsegs, atmo, tels, mk(prec), capacity,
                                    use_cache=not args.no_tune_cache)
        print(f"# autotune precision {prec}: tile_segments={tuned[prec]['tile_segments']} "
              f"waves_per_group={tuned[prec]['waves_per_group']} ({tuned[prec]['ms']:.3f} ms)",
              file=sys.stderr, flush=True)
    ms_mixed, kms_mixed, res_mixed = time_path(hip, ckv, dsegs, atmo, tels,
                                               autotune.apply(mk(ckv.CKV_MIXED), tuned[ckv.CKV_MIXED]),
                                               capacity, args.steps, args.warmup, stream)
    print(f"# mixed: {ms_mixed:.3f} ms/step, bunch kernel {kms_mixed:.3f} ms", file=sys.stderr,
          flush=True)
    ms_fp64, kms_fp64, res_fp64 = time_path(hip, ckv, dsegs, atmo, tels,
                                            autotune.apply(mk(ckv.CKV_FP64), tuned[ckv.CKV_FP64]),
                                            capacity, args.steps, args.warmup, stream)
    print(f"# fp64: {ms_fp64:.3f} ms/step, bunch kernel {kms_fp64:.3f} ms", file=sys.stderr,
          flush=True)
    # the same run with the longitudinal photon-production profile (20 g/cm^2 bins)
    atmo_d = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step,
                            depth=wl.atmo.vertical_depth())
    p_prof = autotune.apply(mk(ckv.CKV_MIXED), tuned[ckv.CKV_MIXED])
    p_prof.depth_bin_gcm2 = PROFILE_BIN_GCM2
    ms_prof, kms_prof, res_prof = time_path(hip, ckv, dsegs, atmo_d, tels, p_prof, capacity,
                                            args.steps, args.warmup, stream)
    print(f"# mixed + profile: {ms_prof:.3f} ms/step, bunch kernel {kms_prof:.3f} ms", file=sys.stderr,
          flush=True)
    # table-lookup ablation: the 57-point profile on its own nodes (binary search per
    # bunch) against the same profile resampled on the 50 m uniform grid
    sp = synth.sparse_atmosphere(wl.atmo.obs_level)
    atmo_n = ckv.Atmosphere(sp.alt, sp.eta, sp.obs_level, nodes=True)
    fine_alt = np.arange(0.0, sp.alt[-1] + 1.0, 50.0)
    atmo_u = ckv.Atmosphere(fine_alt, np.interp(fine_alt, sp.alt, sp.eta), sp.obs_level, 50.0)
    p32 = mk(ckv.CKV_MIXED)
    p32.tile_segments, p32.waves_per_group = 32, tuned[ckv.CKV_MIXED]["waves_per_group"]
    ms_nodes, kms_nodes, res_nodes = time_path(hip, ckv, dsegs, atmo_n, tels, p32, capacity,
                                               args.steps, args.warmup, stream)
    ms_unif, kms_unif, res_unif = time_path(hip, ckv, dsegs, atmo_u, tels, p32, capacity,
                                            args.steps, args.warmup, stream)
    print(f"# node tables (binary search): {ms_nodes:.3f} ms/step; resampled 50 m: {ms_unif:.3f}",
          file=sys.stderr, flush=True)
    for res in (res_mixed, res_fp64, res_prof, res_nodes, res_unif):
        if res["error"] or res["overflow"]:
            raise RuntimeError(f"run reported a problem: {res}")
    nb = res_mixed["n_bunches"]
    assert nb == res_fp64["n_bunches"]
    # untimed: the records of each timed launch, with ids, for the oracle's certificate
    gpu_main = {0: gpu_records(ckv, dsegs, atmo, tels,
                               autotune.apply(mk(ckv.CKV_FP64), tuned[ckv.CKV_FP64]), capacity),
                1: gpu_records(ckv, dsegs, atmo, tels,
                               autotune.apply(mk(ckv.CKV_MIXED), tuned[ckv.CKV_MIXED]), capacity)}
    n_b_main = ckv.count(dsegs, atmo, mk(ckv.CKV_MIXED)).cpu().numpy()
    for prec, r_t in ((0, res_fp64), (1, res_mixed)):
        r_c = gpu_main[prec]["res"]
        if (r_c["n_bunches"], r_c["n_hits"], r_c["drops"]) != (r_t["n_bunches"], r_t["n_hits"],
                                                               r_t["drops"]):
            raise RuntimeError("the certification run differs from the timed run")
    vg_wl, vg_line, vg_recs = vertical_gamma_timing(hip, stream, args.steps, args.warmup)
    print(f"# {vg_wl.name}: {vg_line}", file=sys.stderr, flush=True)

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_probe_mib} MiB read + written, 3 launches", file=sys.stderr)

    k_mixed = emit_kernel_name(1, tuned[ckv.CKV_MIXED]["tile_segments"],
                               tuned[ckv.CKV_MIXED]["waves_per_group"])
    k_fp64 = emit_kernel_name(0, tuned[ckv.CKV_FP64]["tile_segments"],
                              tuned[ckv.CKV_FP64]["waves_per_group"])
    roof = roofline_block(PATH_SLOTS["mixed"], sum(OPS_MIXED.values()), nb, kms_mixed,
                          stored_issue_frac(k_mixed, wl.name))
    roof_fp64 = roofline_block(PATH_SLOTS["fp64"], sum(OPS_FP64.values()), nb, kms_fp64,
                               stored_issue_frac(k_fp64, wl.name))
    roof["traffic"] = stored_traffic("bunch_kernel_single_tev_mixed")
    hits = res_mixed["n_hits"]
    alg_bytes = wl.segs.n * SEG_BYTES + hits * RECORD_BYTES
    line = {
        "metric": "bunches/s gen+propagated, mixed vs FP64 plain at oracle tol; fwd+bwd ms/shower",
        "value": nb / (ms_mixed * 1e-3),
        "unit": "bunches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "steps_in_shower": wl.segs.n, "telescopes": wl.tels.n,
                   "zenith_deg": 20.0, "atmosphere": "5-layer exponential, 50 m grid to 120 km",
                   "bunch_size": wl.bunch_size, "band_nm": [wl.lambda_min, wl.lambda_max],
                   "precision": "mixed",
                   "launch": {"tile_segments": tuned[ckv.CKV_MIXED]["tile_segments"],
                              "waves_per_group": tuned[ckv.CKV_MIXED]["waves_per_group"]}},
        "bunches_per_step": nb,
        "records_per_step": hits,
        "fp64_plain": {"value": nb / (ms_fp64 * 1e-3), "ms_per_step": ms_fp64,
                       "bunch_kernel_ms": kms_fp64,
                       "launch": {"tile_segments": tuned[ckv.CKV_FP64]["tile_segments"],
                                  "waves_per_group": tuned[ckv.CKV_FP64]["waves_per_group"]},
                       "roofline": roof_fp64},
        "mixed_over_fp64": ms_fp64 / ms_mixed,
        "mixed_over_fp64_bunch_kernel": kms_fp64 / kms_mixed,
        "parity": None,
        "vertical_gamma": vg_line,
        "table_ablation": {"profile": "5-layer, 57 tabulated altitudes",
                           "node_tables_binary_search": {"nodes": int(atmo_n.info()[0]),
                                                         "ms_per_step": ms_nodes,
                                                         "bunch_kernel_ms": kms_nodes},
                           "uniform_50m": {"nodes": int(atmo_u.info()[0]), "ms_per_step": ms_unif,
                                           "bunch_kernel_ms": kms_unif},
                           "uniform_over_search": ms_nodes / ms_unif},
        "with_profile": {"bin_gcm2": PROFILE_BIN_GCM2, "bins": atmo_d.profile_bins(PROFILE_BIN_GCM2),
                         "ms_per_step": ms_prof, "bunch_kernel_ms": kms_prof,
                         "value": nb / (ms_prof * 1e-3), "overhead": ms_prof / ms_mixed - 1.0},
        "bunch_kernel_ms": kms_mixed,
        "roofline": roof,
        "hbm": {"algorithmic_bytes_per_launch": alg_bytes,
                "counter_bytes_per_launch": roof["traffic"],
                "achieved_GBs": alg_bytes / (kms_mixed * 1e-3) / 1e9,
                "frac": alg_bytes / (kms_mixed * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "fwd_bwd_ms_per_shower": None,
        "cpu_baseline": None,
    }
    if not args.no_curved:
        line["curved"] = curved_timing(hip, stream)
        torch.cuda.empty_cache()
    if not args.no_diff:
        del dsegs
        torch.cuda.empty_cache()
        d = diff_timing(hip, args.diff_reps)
        print(f"# differentiation: {d}", file=sys.stderr, flush=True)
        line["fwd_bwd_ms_per_shower"] = d["ms_per_shower"]
        line["differentiation"] = d
    if not args.no_batched:
        torch.cuda.empty_cache()
        b = batched_timing(hip, 5, use_cache=not args.no_tune_cache)
        print(f"# batched: {b}", file=sys.stderr, flush=True)
        line["batched"] = b
        torch.cuda.empty_cache()
    samples = []
    if not args.no_streamed:
        line["streamed"], samples = streamed_timing(hip, sample_stride=ZENITH_SAMPLE_STRIDE)
    if args.order_study:
        line["step_order_study"] = order_study(hip, wl, atmo, tels, stream, args.steps, args.warmup)
    ok = True
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["cpu_baseline_one_thread"], par = oracle_leg(wl, gpu_main, n_b_main)
        par["vertical_gamma_every_step"] = oracle_parity_full(vg_wl, vg_recs)
        if samples:
            par["streamed_by_zenith"] = oracle_parity_zeniths(samples, ZENITH_SAMPLE_STRIDE)
        checks = [par["fp64_plain"], par["mixed"], *par["vertical_gamma_every_step"].values(),
                  *par.get("streamed_by_zenith", [])]
        ok = all(c["ok"] for c in checks)
        par["ok"] = ok
        line["parity"] = par
        print(f"# parity: {'green' if ok else 'FAILED'}", file=sys.stderr, flush=True)
    line["device"] = device_info(hip)
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
