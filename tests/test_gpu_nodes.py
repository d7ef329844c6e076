"""Node tables (the profile's own altitudes, binary-search lookups in LDS) in the
bunch kernel, against the oracle's node tables: the table-lookup ablation of the
standard interpolation against the resampled uniform tables."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth

from gpu_helpers import compare_records, gpu_run, say

pytestmark = pytest.mark.gpu


def _sparse_workload(wl):
    atmo = synth.sparse_atmosphere()
    return synth.Workload(wl.name + "_sparse", atmo, wl.tels, wl.segs)


def _node_handles(wl):
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, nodes=True)
    return atmo, ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)


def _cfg(wl):
    t = oracle.build_node_tables(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level)
    return oracle.Config(t, wl.tels.x, wl.tels.y, wl.tels.r, bunch_size=wl.bunch_size,
                         lambda_min=wl.lambda_min, lambda_max=wl.lambda_max, seed=wl.seed)


def test_node_tables_match_oracle():
    wl = _sparse_workload(synth.vertical_gamma(10))
    atmo, _ = _node_handles(wl)
    cfg = _cfg(wl)
    n, h_obs, step = atmo.info()
    assert step == 0.0 and n == cfg.tables.n_nodes
    np.testing.assert_array_equal(atmo.nodes(), cfg.tables.h_nodes)
    psi, P = atmo.tables()
    np.testing.assert_array_equal(psi, cfg.tables.psi)
    np.testing.assert_allclose(P, cfg.tables.P, rtol=1e-13, atol=0)


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_node_tables_vertical_gamma(precision):
    wl = _sparse_workload(synth.vertical_gamma())
    cfg = _cfg(wl)
    r = oracle.run(cfg, wl.segs, nthreads=16)
    g = gpu_run(wl, precision, handles_=_node_handles(wl))
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    say(f"[gpu] node tables vertical gamma prec={precision}: {rep}")


def test_node_tables_hadron_60deg_sampled():
    wl = _sparse_workload(synth.hadron_like(60.0, n_seg=200_000, shower=7))
    cfg = _cfg(wl)
    g = gpu_run(wl, ckv.CKV_MIXED, handles_=_node_handles(wl))
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0
    sd = oracle.segment_details(cfg, wl.segs)
    assert res["n_bunches"] == int(sd["n_b"].sum())
    idx = np.arange(0, wl.segs.n, 13)
    sub = wl.segs.take(idx)
    ores = oracle.run(cfg, sub, nthreads=16, seg_id=idx)
    keep = np.isin(g["ids"][:, 0], idx)
    counts = np.diff(g["offsets"])
    group = np.repeat(np.arange(len(counts)), counts)[keep]
    off = np.zeros_like(g["offsets"])
    off[1:] = np.cumsum(np.bincount(group, minlength=len(counts)))
    rep = compare_records(wl, cfg, ores, dict(offsets=off, rec=g["rec"][keep], ids=g["ids"][keep]),
                          ckv.CKV_MIXED, segs=sub, seg_map=idx)
    say(f"[gpu] node tables hadron 60 deg: {rep}")


def test_node_tables_refuse_other_paths():
    wl = _sparse_workload(synth.vertical_gamma(100))
    atmo, tels = _node_handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    for kw in (dict(tile_segments=16), dict(grazing_exact=True)):
        p = ckv.make_params(precision=ckv.CKV_MIXED, **kw)
        with pytest.raises(ckv.CkvError):
            ckv.Runner(d, atmo, tels, p, 4096).run()
