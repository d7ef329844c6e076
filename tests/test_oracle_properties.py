"""Property tests of the oracle on small random inputs (hypothesis, derandomised so
every run draws the same examples): the refraction series and the exact
cell-by-cell path against the brute-force Snell tracer on random layered
atmospheres, and the sphere test against the closest approach of the ray found
by direct minimisation.  None of the checks reuses the oracle's formulas."""

import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from layer_tracer import C_LIGHT, trace
from paper_2006_14927_amd import synth

PROPS = settings(max_examples=25, deadline=None, derandomize=True,
                 suppress_health_check=[HealthCheck.too_slow])

scale_heights = st.lists(st.floats(5.0, 11.0), min_size=5, max_size=5)


def _config(scales_km, eta0):
    atmo = synth.layered_atmosphere(scales_km=scales_km, eta0=eta0)
    t = oracle.build_tables(atmo.alt, atmo.eta, atmo.obs_level, 50.0)
    grid = t.h_obs + np.arange(t.n_nodes) * t.step
    return oracle.Config(t, [0.0], [0.0], [10.0]), grid, t.psi


def _direction(zen_deg, az_deg):
    th, ph = math.radians(zen_deg), math.radians(az_deg)
    return math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)


@PROPS
@given(scales=scale_heights, eta0=st.floats(2.5e-4, 3.2e-4), zen=st.floats(0.0, 60.0),
       az=st.floats(0.0, 360.0), h_e=st.floats(2300.0, 40_000.0))
def test_series_matches_snell_tracer_on_random_atmospheres(scales, eta0, zen, az, h_e):
    cfg, grid, psi = _config(scales, eta0)
    u, v, w = _direction(zen, az)
    pr = oracle.propagate(cfg, 0.0, 0.0, h_e, u, v, w)
    adv, ct = trace(grid, psi, h_e, math.sin(math.radians(zen)))
    assert math.hypot(pr["x_g"][0], pr["y_g"][0]) == pytest.approx(adv, rel=1e-12, abs=1e-9)
    assert pr["T"][0] == pytest.approx(ct / C_LIGHT, rel=1e-12, abs=1e-8)
    # the displacement lies along the photon's azimuth
    assert pr["x_g"][0] * v - pr["y_g"][0] * u == pytest.approx(0.0, abs=1e-9)


@PROPS
@given(scales=scale_heights, eta0=st.floats(2.5e-4, 3.2e-4), zen=st.floats(0.0, 84.0),
       az=st.floats(0.0, 360.0), h_e=st.floats(2300.0, 40_000.0))
def test_exact_path_matches_snell_tracer_on_random_atmospheres(scales, eta0, zen, az, h_e):
    cfg, grid, psi = _config(scales, eta0)
    u, v, w = _direction(zen, az)
    pr = oracle.propagate_exact(cfg, 0.0, 0.0, h_e, u, v, w)
    adv, ct = trace(grid, psi, h_e, math.sin(math.radians(zen)))
    assert math.hypot(pr["x_g"][0], pr["y_g"][0]) == pytest.approx(adv, rel=1e-11, abs=1e-8)
    assert pr["T"][0] == pytest.approx(ct / C_LIGHT, rel=1e-11, abs=1e-7)


@PROPS
@given(x=st.floats(-50.0, 50.0), y=st.floats(-50.0, 50.0), zen=st.floats(0.0, 80.0),
       az=st.floats(0.0, 360.0), R=st.floats(1.0, 15.0))
def test_sphere_test_is_the_closest_approach(x, y, zen, az, R):
    """Hit iff the observed ray, a line through the ground point, passes within
    R of the sphere centre at the observation level; the distance comes from a
    golden-section search along the line, not from the discriminant."""
    u, v, w = _direction(zen, az)
    X, Y = 3.0, -2.0
    disc = oracle.sphere_disc(x, y, u, v, X, Y, R)

    def dist2(t):
        return (x + t * u - X) ** 2 + (y + t * v - Y) ** 2 + (t * w) ** 2

    lo, hi = -500.0, 500.0
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(200):
        a, b = hi - g * (hi - lo), lo + g * (hi - lo)
        if dist2(a) < dist2(b):
            hi = b
        else:
            lo = a
    d2 = dist2(0.5 * (lo + hi))
    assert disc == pytest.approx(R * R - d2, abs=1e-9 * (1.0 + R * R))
    if abs(R * R - d2) > 1e-6:
        assert (disc >= 0.0) == (d2 <= R * R)
