"""Hadron-like showers (90 % e+-, 10 % muons of 1-100 GeV in a 15 deg cone) at
zenith 0, 20, 40 and 60 deg: the large-zenith muons carry photons with w down
to ~0.25, where the FP32 parts of the mixed path have the least margin."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth

from gpu_helpers import compare_records, gpu_run, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("zenith", [0.0, 20.0, 40.0, 60.0])
@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_hadron_like_parity(zenith, precision):
    wl = synth.hadron_like(zenith, n_seg=40_000, shower=int(zenith))
    cfg = oracle.Config.from_workload(wl)
    r = oracle.run(cfg, wl.segs, nthreads=16)
    g = gpu_run(wl, precision)
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    say(f"[gpu] hadron_like zenith={zenith} prec={precision}: bunches={res['n_bunches']} {rep}")


def test_all_candidate_levels_and_all_sphere_path():
    """Showers from 0 to 80 deg zenith with half the steps from muons in a 15 deg
    cone: crossings arrive with observed w on both sides of every candidate-grid
    level (0.2, 0.5, 0.85), and below 0.2, where every sphere is tested."""
    atmo = synth.layered_atmosphere()
    parts = [synth.shower_segments(i, 15_000, atmo, zenith_deg=z, xmax=500.0, muon_fraction=0.5,
                                   shower_id=i)
             for i, z in enumerate((0.0, 30.0, 50.0, 65.0, 75.0, 80.0))]
    wl = synth.Workload("zenith_mix", atmo, synth.telescopes_disk(), synth.Segments.concat(parts))
    cfg = oracle.Config.from_workload(wl)
    r = oracle.run(cfg, wl.segs, nthreads=16)
    rec = r.rec
    w_obs = np.sqrt(np.maximum(0.0, 1.0 - rec[:, 2] ** 2 - rec[:, 3] ** 2))
    bands = np.histogram(w_obs, bins=[0.0, 0.2, 0.5, 0.85, 1.0])[0]
    say(f"[gpu] zenith mix: hits per observed-w band {bands.tolist()}")
    assert (bands > 0).all()
    for precision in (ckv.CKV_FP64, ckv.CKV_MIXED):
        g = gpu_run(wl, precision)
        res = g["result"]
        assert res["error"] == 0 and res["overflow"] == 0
        assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops
        if precision == ckv.CKV_FP64:
            np.testing.assert_array_equal(g["offsets"], r.offsets)
        rep = compare_records(wl, cfg, r, g, precision)
        say(f"[gpu] zenith mix prec={precision}: {rep}")
