"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare its records with the FP64 oracle."""

import sys

import numpy as np

import oracle
from paper_2006_14927_amd import ckv

# tolerances of the mixed-precision path against the FP64 oracle
TOL_GROUND_M = 1e-3        # dx, dy
TOL_DIR = 1e-6             # u_obs, v_obs
TOL_T_NS = 0.01            # arrival time
TOL_REL = 1e-6             # photons, lambda (relative)
GUARD_EPS_M = 1e-3         # hit decisions may differ when |disc| <= 2 R eps + eps^2
F32 = 2.0 ** -24           # half an FP32 ulp, relative


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def handles(wl):
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    return atmo, tels


def params(wl, precision, **kw):
    return ckv.make_params(precision=precision, bunch_size=wl.bunch_size, lambda_min=wl.lambda_min,
                           lambda_max=wl.lambda_max, seed=wl.seed, **kw)


def gpu_run(wl, precision, *, segs=None, capacity=None, seg_id_base=None, handles_=None,
            want_ids=True, **kw):
    import torch
    segs = wl.segs if segs is None else segs
    atmo, tels = handles_ if handles_ is not None else handles(wl)
    d = ckv.DeviceSegments(segs, seg_id_base=seg_id_base)
    p = params(wl, precision, **kw)
    cap = capacity if capacity is not None else max(1024, segs.n * 4)
    say(f"[gpu] run {wl.name} n={segs.n} showers={segs.n_showers} prec={precision} cap={cap} {kw}")
    r = ckv.Runner(d, atmo, tels, p, cap, want_ids=want_ids)
    out = r.run()
    torch.cuda.synchronize()
    res = out.result()
    if res["overflow"] and capacity is None:
        cap = int(res["n_hits"]) + 16
        say(f"[gpu] rerun with capacity {cap}")
        r = ckv.Runner(d, atmo, tels, p, cap, want_ids=want_ids)
        out = r.run()
        torch.cuda.synchronize()
        res = out.result()
    n = int(res["n_records"])
    return dict(offsets=out.tel_offsets.cpu().numpy(), rec=out.records[:n].cpu().numpy(),
                ids=out.ids[:n].cpu().numpy() if want_ids else None, result=res)


def group_keys(offsets, seg, k, n_seg_max, k_max):
    counts = np.diff(offsets)
    group = np.repeat(np.arange(len(counts), dtype=np.int64), counts)
    return (group * (n_seg_max + 1) + seg.astype(np.int64)) * (k_max + 1) + k.astype(np.int64), group


def compare_records(wl, cfg, ores, g, precision, *, segs=None, seg_map=None):
    """Check GPU records against oracle hits.

    seg_map maps oracle segment indices to the GPU's (for subset runs)."""
    segs = wl.segs if segs is None else segs
    n_tel = cfg.n_tel
    o_seg = ores.seg if seg_map is None else seg_map[ores.seg]
    n_seg_max = int(max(o_seg.max(initial=0), g["ids"][:, 0].max(initial=0))) + 1
    k_max = int(max(ores.k.max(initial=0), g["ids"][:, 1].max(initial=0))) + 1
    ok, ogroup = group_keys(ores.offsets, o_seg, ores.k, n_seg_max, k_max)
    gk, ggroup = group_keys(g["offsets"], g["ids"][:, 0], g["ids"][:, 1], n_seg_max, k_max)
    # canonical order: groups ascending, then (step, bunch) ascending
    assert np.all(np.diff(gk) > 0), "GPU records out of canonical order"
    assert np.all(np.diff(ok) > 0)
    common, io, ig = np.intersect1d(ok, gk, assume_unique=True, return_indices=True)
    only_o = np.setdiff1d(np.arange(len(ok)), io)
    only_g = np.setdiff1d(np.arange(len(gk)), ig)
    ro, rg = ores.rec[io], g["rec"][ig].astype(np.float64)
    report = dict(matched=len(common), only_oracle=len(only_o), only_gpu=len(only_g))
    if precision == ckv.CKV_FP64:
        assert len(only_o) == 0 and len(only_g) == 0, report
        # FP64 path: records equal the oracle up to the final FP32 rounding
        tol = 2 * F32 * np.abs(ro) + 1e-9
        tol[:, 4] += 2e-7           # time is accumulated over ~1e5 ns before t_ref
        bad = np.abs(rg - ro) > tol
        assert not bad.any(), (report, np.argwhere(bad)[:5], (rg - ro)[bad][:5])
    else:
        tel_r = cfg.tr
        guard = lambda tel: 2 * tel_r[tel] * GUARD_EPS_M + GUARD_EPS_M ** 2
        tel_o = (ogroup[only_o] % n_tel)
        assert np.all(np.abs(ores.disc[only_o]) <= guard(tel_o)), report
        if len(only_g):
            tel_g = ggroup[only_g] % n_tel
            gs = g["ids"][only_g, 0]
            inv = {v: i for i, v in enumerate(seg_map)} if seg_map is not None else None
            osg = np.array([inv[x] for x in gs]) if inv else gs
            bd = oracle.bunch_details(cfg, segs, osg, g["ids"][only_g, 1])
            disc = np.array([oracle.sphere_disc(bd["x_g"][i], bd["y_g"][i], bd["u_o"][i], bd["v_o"][i],
                                                cfg.tx[t], cfg.ty[t], cfg.tr[t])
                             for i, t in enumerate(tel_g)])
            assert np.all(np.abs(disc) <= guard(tel_g)), report
        d = np.abs(rg - ro)
        report.update(max_ground=float(d[:, :2].max(initial=0)), max_dir=float(d[:, 2:4].max(initial=0)),
                      max_t=float(d[:, 4].max(initial=0)))
        assert d[:, :2].max(initial=0) <= TOL_GROUND_M, report
        assert d[:, 2:4].max(initial=0) <= TOL_DIR, report
        assert d[:, 4].max(initial=0) <= TOL_T_NS, report
        assert np.all(d[:, 5] <= 2 * F32 * np.abs(ro[:, 5]) + 1e-6), report
        assert np.all(d[:, 6] <= TOL_REL * np.abs(ro[:, 6])), report
        assert np.all(d[:, 7] <= TOL_REL * np.abs(ro[:, 7])), report
    return report
