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
