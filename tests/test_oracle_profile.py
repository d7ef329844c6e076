"""Pins of the oracle's longitudinal photon-production profile (photons and bunches
per bin of vertical depth of the emission point, per shower): the depth table
against the tabulated thickness and a closed form, the binning against a brute
force over the oracle's own bunch records (numpy interpolation and histogram),
a vertical step in a constant-density atmosphere against the uniform spread of
its sub-steps, and the total against the Frank-Tamm yield of the steps."""

import math

import numpy as np

import oracle
from paper_2006_14927_amd import synth


def _vg(n=400):
    wl = synth.vertical_gamma(n)
    cfg = oracle.Config.from_workload(wl)
    T = oracle.build_depth(wl.atmo.alt, wl.atmo.vertical_depth(), cfg.tables)
    return wl, cfg, T


def test_depth_table_nodes_and_closed_form():
    wl, cfg, T = _vg(10)
    grid = cfg.tables.h_obs + np.arange(cfg.tables.n_nodes) * cfg.tables.step
    # grid nodes coincide with the 100 m input nodes: values taken exactly
    depth = wl.atmo.vertical_depth()
    idx = np.searchsorted(wl.atmo.alt, grid)
    np.testing.assert_array_equal(T, depth[idx])
    # exponential density: X(h) = X(0) exp(-h / H) (+ the part above the table)
    H = 8400.0
    x0 = 2.9e-4 * (1.225e-3 / 2.9e-4) * H * 100.0
    np.testing.assert_allclose(T, x0 * np.exp(-grid / H), rtol=2e-5)
    # a table node off the grid is interpolated linearly in altitude
    alt = np.array([0.0, 1000.0, 5000.0, 20000.0])
    d = np.array([1000.0, 900.0, 500.0, 100.0])
    t = oracle.Tables(1000.0, 1500.0, np.zeros(12), np.zeros((5, 12)))
    got = oracle.build_depth(alt, d, t)
    want = np.interp(1000.0 + 1500.0 * np.arange(12), alt, d)
    np.testing.assert_allclose(got, want, rtol=1e-15)


def test_profile_equals_brute_force_binning():
    wl, cfg, T = _vg(400)
    width = 20.0
    ph, bu = oracle.profile(cfg, wl.segs, T, width, nthreads=4)
    sd = oracle.segment_details(cfg, wl.segs)
    nb = sd["n_b"].astype(np.int64)
    seg = np.repeat(np.arange(wl.segs.n), nb)
    k = np.concatenate([np.arange(n) for n in nb])
    bd = oracle.bunch_details(cfg, wl.segs, seg, k)
    grid = cfg.tables.h_obs + np.arange(cfg.tables.n_nodes) * cfg.tables.step
    inside = (bd["h_e"] >= grid[0]) & (bd["h_e"] < grid[-1])
    X = np.interp(bd["h_e"][inside], grid, T)
    edges = np.arange(ph.shape[1] + 1) * width
    cnt, _ = np.histogram(X, bins=edges)
    w, _ = np.histogram(X, bins=edges, weights=bd["photons"][inside])
    # bunches within rounding of a bin edge may fall either way
    near = np.abs(X / width - np.round(X / width)) < 1e-9
    assert near.sum() == 0
    np.testing.assert_array_equal(bu[0], cnt)
    np.testing.assert_allclose(ph[0], w, rtol=1e-12, atol=1e-9)
    assert bu.sum() == inside.sum() > 10_000


def test_vertical_step_in_constant_density():
    """rho constant: X is linear in altitude, so a vertical step spreads its
    n_b bunches over the depth bins in proportion to the altitude overlap: one
    bunch per equal sub-step, so a bin holds its whole sub-steps plus 0 or 1
    from each of the two it cuts, i.e. within 2 of n_b x overlap / L."""
    alt = np.arange(0.0, 30001.0, 100.0)
    eta = np.full(alt.shape, 2.0e-4)
    rho = 1.0e-3                                     # g/cm^3
    depth = rho * (30000.0 - alt) * 100.0            # g/cm^2
    tels = synth.telescopes_grid()
    t = oracle.build_tables(alt, eta, 2000.0, 50.0)
    cfg = oracle.Config(t, tels.x, tels.y, tels.r)
    T = oracle.build_depth(alt, depth, t)
    L, h0 = 3000.0, 15000.0
    segs = synth.Segments(np.zeros(1), np.zeros(1), np.full(1, h0), np.zeros(1), np.zeros(1),
                          np.ones(1), np.full(1, L), np.zeros(1), np.full(1, 5.0e4),
                          np.zeros(1, np.uint8), np.array([0, 1]), np.zeros(1),
                          np.zeros(1, np.uint32))
    width = 10.0
    ph, bu = oracle.profile(cfg, segs, T, width)
    n_b = int(oracle.segment_details(cfg, segs)["n_b"][0])
    assert bu.sum() == n_b > 500
    edges_x = np.arange(bu.shape[1] + 1) * width
    edges_h = 30000.0 - edges_x / (rho * 100.0)      # altitude of each depth edge
    lo = np.maximum(np.minimum(edges_h[:-1], h0), h0 - L)
    hi = np.maximum(np.minimum(edges_h[1:], h0), h0 - L)
    expect = n_b * (lo - hi) / L
    assert np.all(np.abs(bu[0] - expect) < 2.0)
    assert np.abs(bu[0] - expect).max() > 0.5           # the test can see a shift


def test_total_equals_frank_tamm_yield_and_showers_separate():
    wl, cfg, T = _vg(300)
    sd = oracle.segment_details(cfg, wl.segs)
    ph, bu = oracle.profile(cfg, wl.segs, T, 25.0, nthreads=3)
    assert math.isclose(ph.sum(), sd["N"][sd["status"] == -1].sum(), rel_tol=1e-12)
    assert bu.sum() == int(sd["n_b"].sum())
    # two showers: each keeps its own row
    two = synth.Segments.concat([wl.segs.take(np.arange(0, 120)), wl.segs.take(np.arange(120, 300))])
    two.shower_ids[:] = 0                              # same random numbers as the one-shower run
    p2, b2 = oracle.profile(cfg, two, T, 25.0, seg_id_base=[0, 120])
    np.testing.assert_array_equal(b2.sum(axis=0), bu[0])
    np.testing.assert_allclose(p2.sum(axis=0), ph[0], rtol=1e-12)
    p_a, b_a = oracle.profile(cfg, wl.segs.take(np.arange(0, 120)), T, 25.0)
    np.testing.assert_array_equal(b2[0], b_a[0])
