"""Pins of the oracle's differentiation pieces: the soft response against a
direct evaluation with scipy's normal CDF, the parameterised atmosphere
against closed forms, and finite differences of the travel time against the
analytic derivative for a vertical ray."""

import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2006_14927_amd import synth

C_LIGHT = 0.299792458


def _spec(dw):
    return oracle.AtmoParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level,
                                dw.step, dw.top)


def test_param_profile_closed_forms():
    dw = synth.diff_showers(1, 10)
    spec = _spec(dw)
    h = np.linspace(2200.0, 119000.0, 57)
    # equal scale heights and zero knots: a single exponential
    th = np.concatenate([np.zeros(dw.n_knots), np.full(8, 8000.0)])
    np.testing.assert_allclose(oracle.eta_from_params(spec, th, h), 2.9e-4 * np.exp(-h / 8000.0),
                               rtol=1e-13)
    # knots only (scale heights huge): log eta = log eta0 + linear interpolant of the knots
    rng = np.random.default_rng(1)
    kn = rng.normal(0, 0.1, dw.n_knots)
    th = np.concatenate([kn, np.full(8, 1e30)])
    hk = np.arange(dw.n_knots) * dw.knot_top / (dw.n_knots - 1)
    ref = math.log(2.9e-4) + np.interp(np.minimum(h, dw.knot_top), hk, kn)
    np.testing.assert_allclose(np.log(oracle.eta_from_params(spec, th, h)), ref, rtol=0, atol=1e-12)
    # layered scale heights: depth is the piecewise sum of overlaps / H_l
    th = dw.theta0
    b = dw.layer_bounds
    Hs = th[dw.n_knots:]
    depth = sum(np.clip(np.minimum(h, b[l + 1] if l < 7 else np.inf) - b[l], 0, None) / Hs[l]
                for l in range(8))
    np.testing.assert_allclose(oracle.eta_from_params(spec, th, h), 2.9e-4 * np.exp(-depth), rtol=1e-13)


def test_soft_response_matches_direct_normal_cdf():
    dw = synth.diff_showers(1, 400)
    spec = _spec(dw)
    t = oracle.tables_from_params(spec, dw.theta0)
    cfg = oracle.Config(t, dw.tels.x, dw.tels.y, dw.tels.r, seed=dw.seed)
    sd = oracle.segment_details(cfg, dw.segs)
    nb = sd["n_b"].astype(np.int64)
    S, A = oracle.soft(cfg, dw.segs, nb, dw.sigma)
    # direct: every bunch, every telescope, scipy's normal CDF
    seg = np.repeat(np.arange(dw.segs.n), nb)
    k = np.concatenate([np.arange(n) for n in nb])
    bd = oracle.bunch_details(cfg, dw.segs, seg, k)
    ok = bd["status"] == -1
    Sd = np.zeros(dw.tels.n)
    Ad = np.zeros(dw.tels.n)
    for q in range(dw.tels.n):
        dx = bd["x_g"][ok] - dw.tels.x[q]
        dy = bd["y_g"][ok] - dw.tels.y[q]
        b = dx * bd["u_o"][ok] + dy * bd["v_o"][ok]
        rho2 = dx * dx + dy * dy - b * b
        R = dw.tels.r[q]
        W = stats.norm.cdf((R * R - rho2) / (2 * R * dw.sigma))
        Sd[q] = np.sum(bd["photons"][ok] * W)
        Ad[q] = np.sum(bd["photons"][ok] * W * bd["t"][ok])
    assert Sd.sum() > 10
    np.testing.assert_allclose(S[0], Sd, rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(A[0], Ad, rtol=1e-11, atol=1e-300)


def test_vertical_travel_time_derivative_by_finite_differences():
    """dT/dpsi_i for a vertical ray = (1/c) int hat_i(h) / (2 n(h)) dh (hat: the
    linear interpolation weight of node i); finite differences of the oracle's
    propagation against this closed form."""
    atmo = synth.exponential_atmosphere(step=100.0, h_max=30000.0)
    t = oracle.build_tables(atmo.alt, atmo.eta, 2200.0)
    grid = 2200.0 + np.arange(t.n_nodes) * 100.0
    h_e = 9876.5
    x, wts = np.polynomial.legendre.leggauss(10)
    for i in (3, 40, 76):
        # closed form by Gauss quadrature of hat_i / (2 n) over the cells around node i
        ref = 0.0
        for a_, b_ in ((grid[i - 1], grid[i]), (grid[i], grid[i + 1])):
            hi = min(b_, h_e)
            if hi <= a_:
                continue
            z = a_ + (hi - a_) * 0.5 * (x + 1)
            hat = np.interp(z, grid, (np.arange(t.n_nodes) == i).astype(float))
            n = np.sqrt(1 + np.interp(z, grid, t.psi))
            ref += 0.5 * (hi - a_) * np.sum(wts * hat / (2 * n))
        ref /= C_LIGHT

        def T_of(dpsi):
            psi = t.psi.copy()
            psi[i] += dpsi
            # moments of the perturbed profile (exact cell integrals)
            P = np.zeros_like(t.P)
            for j in range(1, 6):
                cell = [100.0 / (j + 1) * sum(psi[c] ** (j - m) * psi[c + 1] ** m for m in range(j + 1))
                        for c in range(len(psi) - 1)]
                P[j - 1, 1:] = np.cumsum(cell)
            cfg = oracle.Config(oracle.Tables(2200.0, 100.0, psi, P), [0.0], [0.0], [10.0])
            return oracle.propagate(cfg, 0.0, 0.0, h_e, 0.0, 0.0, 1.0)["T"][0]

        d = 1e-3 * t.psi[i]
        fd = (T_of(d) - T_of(-d)) / (2 * d)
        assert fd == pytest.approx(ref, rel=1e-6)
