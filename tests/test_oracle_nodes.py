"""Pins of the oracle's node tables: the standard interpolation on the input's own
(non-uniform) altitudes with a binary search (the RPOL way), as opposed to the
resampled uniform tables.  Against quadrature of the piecewise-linear psi, the
brute-force layer tracer on the same nodes, and the uniform tables where both
describe the same function."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import synth

from layer_tracer import C_LIGHT, trace


def _gauss(grid, psi, lo, hi, fn, npts=8):
    x, wts = np.polynomial.legendre.leggauss(npts)
    edges = np.concatenate([[lo], grid[(grid > lo) & (grid < hi)], [hi]])
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        z = 0.5 * (b - a) * x + 0.5 * (a + b)
        total += 0.5 * (b - a) * np.sum(wts * fn(np.interp(z, grid, psi)))
    return total


def _sparse():
    atmo = synth.sparse_atmosphere()
    t = oracle.build_node_tables(atmo.alt, atmo.eta, atmo.obs_level)
    tels = synth.telescopes_grid()
    return atmo, t, oracle.Config(t, tels.x, tels.y, tels.r)


def test_node_tables_nodes_and_moments():
    atmo, t, cfg = _sparse()
    hn = t.h_nodes
    assert hn[0] == 2200.0 and np.all(np.diff(hn) > 0) and hn[-1] == 120000.0
    assert 50 <= t.n_nodes <= 60
    eta = np.interp(hn, atmo.alt, atmo.eta)
    np.testing.assert_allclose(t.psi, np.expm1(2 * np.log1p(eta)), rtol=1e-13)
    for j in range(1, 6):
        for i in (1, 7, 20, t.n_nodes - 1):
            want = _gauss(hn, t.psi, hn[0], hn[i], lambda p: p ** j)
            np.testing.assert_allclose(t.P[j - 1, i], want, rtol=1e-12)


def test_node_lookup_by_search():
    atmo, t, cfg = _sparse()
    hn = t.h_nodes
    rng = np.random.default_rng(3)
    h = np.concatenate([hn[:-1], rng.uniform(hn[0], hn[-1], 300)])
    out = oracle.lookup(cfg, h)
    np.testing.assert_allclose(out[:, 0], np.interp(h, hn, t.psi), rtol=1e-14)
    for q in range(0, len(h), 37):
        for j in range(1, 6):
            want = _gauss(hn, t.psi, hn[0], h[q], lambda p: p ** j)
            np.testing.assert_allclose(out[q, j], want, rtol=1e-11, atol=1e-300)


@pytest.mark.parametrize("zenith_deg", [5.0, 30.0, 60.0])
def test_node_tables_against_layer_tracer(zenith_deg):
    atmo, t, cfg = _sparse()
    s = np.sin(np.radians(zenith_deg))
    w = np.cos(np.radians(zenith_deg))
    for h_e in (3000.0, 8123.4, 17500.0, 29999.0):
        r = oracle.propagate(cfg, 0.0, 0.0, h_e, s, 0.0, w)
        adv, ct = trace(t.h_nodes, t.psi, h_e, s)
        assert abs(r["x_g"][0] - adv) <= 1e-9 + 1e-12 * adv
        assert abs(r["T"][0] * C_LIGHT - ct) <= 1e-8
        e = oracle.propagate_exact(cfg, 0.0, 0.0, h_e, s, 0.0, w)
        np.testing.assert_allclose(e["x_g"][0], adv, rtol=1e-12, atol=1e-12)


def test_node_tables_equal_uniform_tables_on_a_uniform_input():
    wl = synth.vertical_gamma(2000)
    a = wl.atmo
    tu = oracle.build_tables(a.alt, a.eta, a.obs_level, 0.0)
    tn = oracle.build_node_tables(a.alt, a.eta, a.obs_level)
    np.testing.assert_array_equal(tn.h_nodes, tu.grid())
    np.testing.assert_array_equal(tn.psi, tu.psi)
    np.testing.assert_allclose(tn.P, tu.P, rtol=1e-14, atol=0)
    cu = oracle.Config(tu, wl.tels.x, wl.tels.y, wl.tels.r)
    cn = oracle.Config(tn, wl.tels.x, wl.tels.y, wl.tels.r)
    ru = oracle.run(cu, wl.segs, nthreads=4)
    rn = oracle.run(cn, wl.segs, nthreads=4)
    assert ru.n_bunches == rn.n_bunches and ru.drops == rn.drops
    np.testing.assert_array_equal(ru.offsets, rn.offsets)
    np.testing.assert_allclose(rn.rec, ru.rec, rtol=1e-12, atol=1e-9)


def test_uniform_resampling_converges_to_node_tables():
    """Accuracy against table size: the uniform tables resample the 57-point
    profile onto grids whose nodes miss its kinks; their ground points and
    times approach the node tables' as the step shrinks, to ~1e-5 m and
    ~2e-5 ns at ~10 000 points (the paper's fast-table size, sec. 3.3.2)."""
    atmo, tn, cn = _sparse()
    rng = np.random.default_rng(9)
    m = 400
    th = np.radians(rng.uniform(0, 60, m))
    h = rng.uniform(3000, 30000, m)
    args = (0.0, 0.0, h, np.sin(th), 0.0, np.cos(th))
    ref = oracle.propagate(cn, *args)
    errs = []
    for step in (170.0, 70.0, 17.0, 11.9):
        alt = np.arange(0.0, 120000.0 + 1, step)
        tu = oracle.build_tables(alt, np.interp(alt, atmo.alt, atmo.eta), atmo.obs_level, step)
        cu = oracle.Config(tu, cn.tx, cn.ty, cn.tr)
        r = oracle.propagate(cu, *args)
        errs.append((tu.n_nodes, np.abs(r["x_g"] - ref["x_g"]).max(), np.abs(r["T"] - ref["T"]).max()))
    for a, b in zip(errs[:-1], errs[1:]):
        assert a[1] > b[1] and a[2] > b[2], errs
    assert errs[-1][0] > 9000 and errs[-1][1] < 2e-5 and errs[-1][2] < 1e-4, errs
    assert errs[0][1] > 5e-4                       # the coarse table is visibly off
