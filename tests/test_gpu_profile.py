"""Longitudinal photon-production profile (photons and bunches per bin of
vertical depth of the emission point, per shower) computed inside the bunch
kernel, against the oracle: bunch counts bit-exact, photon sums to FP64
rounding, the records of the run unchanged by it."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth

from gpu_helpers import params, say

pytestmark = pytest.mark.gpu

PRECISIONS = [ckv.CKV_FP64, ckv.CKV_MIXED]


def _handles(wl):
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step,
                          depth=wl.atmo.vertical_depth())
    return atmo, ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)


def _oracle(wl, width, segs=None, **kw):
    cfg = oracle.Config.from_workload(wl)
    T = oracle.build_depth(wl.atmo.alt, wl.atmo.vertical_depth(), cfg.tables)
    ph, bu = oracle.profile(cfg, wl.segs if segs is None else segs, T, width, nthreads=16, **kw)
    return cfg, T, ph, bu


def _run(wl, atmo, tels, precision, width, capacity=None, **kw):
    import torch
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, precision, depth_bin=width, **kw)
    r = ckv.Runner(d, atmo, tels, p, capacity or max(4096, 4 * wl.segs.n))
    out = r.run()
    torch.cuda.synchronize()
    res = out.result()
    assert res["error"] == 0 and res["overflow"] == 0
    n = res["n_records"]
    return (out.profile_photons.cpu().numpy(), out.profile_bunches.cpu().numpy(),
            out.records[:n].cpu().numpy(), out.tel_offsets.cpu().numpy(), res)


def test_depth_table_matches_oracle():
    for wl in (synth.vertical_gamma(10), synth.single_tev(10)):
        atmo, _ = _handles(wl)
        cfg, T, _, _ = _oracle(wl, 20.0, segs=wl.segs)
        np.testing.assert_array_equal(atmo.depth(), T)
        assert atmo.profile_bins(20.0) == oracle.profile_bins(T, 20.0)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_profile_vertical_gamma(precision):
    wl = synth.vertical_gamma()
    atmo, tels = _handles(wl)
    _, _, ph_o, bu_o = _oracle(wl, 10.0)
    ph, bu, rec, off, res = _run(wl, atmo, tels, precision, 10.0)
    np.testing.assert_array_equal(bu, bu_o)
    np.testing.assert_allclose(ph, ph_o, rtol=1e-12, atol=1e-9)
    assert bu.sum() == res["n_bunches"] > 900_000
    # the records do not depend on the profile
    import torch
    d = ckv.DeviceSegments(wl.segs)
    out = ckv.Runner(d, atmo, tels, params(wl, precision), max(4096, 4 * wl.segs.n)).run()
    torch.cuda.synchronize()
    n = out.result()["n_records"]
    np.testing.assert_array_equal(out.tel_offsets.cpu().numpy(), off)
    np.testing.assert_array_equal(out.records[:n].cpu().numpy().view(np.uint32), rec.view(np.uint32))
    say(f"[gpu] profile vertical gamma prec={precision}: {bu.shape[1]} bins, {bu.sum()} bunches")


def test_profile_single_tev_full_size():
    wl = synth.single_tev()
    atmo, tels = _handles(wl)
    _, _, ph_o, bu_o = _oracle(wl, 20.0)
    ph, bu, _, _, res = _run(wl, atmo, tels, ckv.CKV_MIXED, 20.0, capacity=4_000_000)
    np.testing.assert_array_equal(bu, bu_o)
    np.testing.assert_allclose(ph, ph_o, rtol=1e-12, atol=1e-9)
    say(f"[gpu] profile single TeV: {bu.sum()} bunches in {bu.shape[1]} bins, "
        f"peak bin {int(np.argmax(ph[0]))}")


def test_profile_batched_tilings_and_graph():
    import torch
    wl = synth.batched_showers(256, seg_scale=5e-4)
    atmo, tels = _handles(wl)
    _, _, ph_o, bu_o = _oracle(wl, 25.0)
    base = None
    for kw in (dict(), dict(tile_segments=16), dict(tile_segments=64, waves_per_group=8)):
        ph, bu, _, _, _ = _run(wl, atmo, tels, ckv.CKV_MIXED, 25.0, **kw)
        np.testing.assert_array_equal(bu, bu_o)
        np.testing.assert_allclose(ph, ph_o, rtol=1e-12, atol=1e-9)
        base = base if base is not None else bu
    d = ckv.DeviceSegments(wl.segs)
    gr = ckv.GraphRunner(ckv.Runner(d, atmo, tels, params(wl, ckv.CKV_MIXED, depth_bin=25.0),
                                    max(4096, 4 * wl.segs.n)))
    for rep in range(3):
        gr.runner.profile_bunches.fill_(-1)
        gr.runner.profile_photons.fill_(float("nan"))
        torch.cuda.synchronize()
        out = gr.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.profile_bunches.cpu().numpy(), bu_o)
        np.testing.assert_allclose(out.profile_photons.cpu().numpy(), ph_o, rtol=1e-12, atol=1e-9)
    say(f"[gpu] profile batched: {wl.segs.n_showers} showers x {bu_o.shape[1]} bins")


def test_profile_requires_depth_table():
    wl = synth.vertical_gamma(100)
    atmo = ckv.Atmosphere(wl.atmo.alt, wl.atmo.eta, wl.atmo.obs_level, wl.fine_step)
    tels = ckv.TelescopeArray(wl.tels.x, wl.tels.y, wl.tels.r)
    d = ckv.DeviceSegments(wl.segs)
    with pytest.raises(ckv.CkvError):
        ckv.Runner(d, atmo, tels, params(wl, ckv.CKV_MIXED, depth_bin=10.0), 4096)
    atmo2, _ = _handles(wl)
    with pytest.raises(ckv.CkvError):
        atmo2.profile_bins(1.0)          # more than CKV_MAX_PROFILE_BINS bins


@pytest.mark.parametrize("precision", PRECISIONS)
def test_profile_near_maximum_bins(precision):
    """6.25 g/cm^2 bins: 127 of the CKV_MAX_PROFILE_BINS = 128 histogram slots."""
    wl = synth.vertical_gamma(4000)
    atmo, tels = _handles(wl)
    assert atmo.profile_bins(6.25) == 127
    _, _, ph_o, bu_o = _oracle(wl, 6.25)
    ph, bu, _, _, _ = _run(wl, atmo, tels, precision, 6.25)
    np.testing.assert_array_equal(bu, bu_o)
    np.testing.assert_allclose(ph, ph_o, rtol=1e-12, atol=1e-9)
