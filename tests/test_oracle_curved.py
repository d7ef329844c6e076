"""Pins of the oracle's curved-atmosphere variant (spherical shells; every
bunch traced exactly): the brute-force shell tracer (straight lines between
spheres and vector Snell refraction, `tests/sphere_tracer.py`), a uniform
medium (a straight chord to the observation sphere), a radial ray, the limit of
a very large radius (the plane-parallel exact path), and the run-level switch."""

import math

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import synth

from sphere_tracer import C_LIGHT, trace, trace_extrapolated

R_EARTH = 6371000.0


def _cfg(R=R_EARTH, wl=None, **kw):
    atmo = synth.layered_atmosphere()
    t = oracle.build_tables(atmo.alt, atmo.eta, atmo.obs_level, 50.0)
    tels = synth.telescopes_grid()
    return t, oracle.Config(t, tels.x, tels.y, tels.r, earth_radius=R, **kw)


def test_altitude_of_a_point():
    for (x, y, z) in [(0.0, 0.0, 5000.0), (1000.0, -300.0, 2200.0), (1e5, 2e5, 15000.0),
                      (-3e5, 0.0, 100.0), (0.0, 0.0, 0.0)]:
        want = np.sqrt(np.longdouble(x) ** 2 + np.longdouble(y) ** 2 +
                       (np.longdouble(R_EARTH) + np.longdouble(z)) ** 2) - np.longdouble(R_EARTH)
        got = oracle.curved_altitude(R_EARTH, x, y, z)
        assert abs(got - float(want)) <= 1e-9 * max(1.0, abs(float(want)))
    assert oracle.curved_altitude(R_EARTH, 0.0, 0.0, 4321.5) == 4321.5


CASES = [  # zenith [deg], azimuth [deg], emission z [m], x [m], y [m]
    (0.0, 0.0, 10000.0, 0.0, 0.0),
    (20.0, 30.0, 8000.0, 500.0, -200.0),
    (45.0, 200.0, 25000.0, -8000.0, 3000.0),
    (60.0, 0.0, 12000.0, 5000.0, 300.0),
    (70.0, 90.0, 30000.0, 0.0, -40000.0),
    (75.0, 180.0, 15000.0, -30000.0, 300.0),
    (80.0, 0.0, 9000.0, -60000.0, 0.0),
    (84.0, 0.0, 20000.0, -150000.0, 2000.0),
]


@pytest.mark.parametrize("zen,az,z,x,y", CASES)
def test_against_shell_tracer(zen, az, z, x, y):
    t, cfg = _cfg()
    th, ph = math.radians(zen), math.radians(az)
    D = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th))
    o = oracle.propagate_curved(cfg, x, y, z, D[0], D[1], -D[2])
    ref = trace_extrapolated(R_EARTH, t.grid(), t.psi, t.h_obs, (x, y, z), D, m=8)
    assert o["status"][0] == -1 and ref is not None
    xg, yg, uo, vo, T = ref
    # the tracer's own rounding: ~1e-9 m per step on coordinates of size R
    # over up to 3e4 steps, i.e. ~1e-12 of the path
    path = T * C_LIGHT
    assert abs(o["x_g"][0] - xg) < 2e-7 + 2e-12 * path and abs(o["y_g"][0] - yg) < 2e-7 + 2e-12 * path
    assert abs(o["u_o"][0] - uo) < 1e-12 and abs(o["v_o"][0] - vo) < 1e-12
    assert abs(o["T"][0] - T) < 1e-7 + 2e-12 * T
    # Bouguer invariant: n_obs r_obs sin(zeta_g) = n_e r_e sin(zeta_e)
    assert abs(o["w_o"][0] ** 2 + o["u_o"][0] ** 2 + o["v_o"][0] ** 2 - 1.0) < 1e-14


def test_turning_and_upward_rays():
    t, cfg = _cfg()
    # 85.9 deg from the local vertical at 20 km: above the 2.2 km sphere's dip, turns
    th = math.radians(85.0)
    D = (math.sin(th), 0.0, -math.cos(th))
    o = oracle.propagate_curved(cfg, 100000.0, 0.0, 20000.0, D[0], D[1], -D[2])
    assert o["status"][0] == oracle.DROP_NAMES.index("grazing")
    assert trace(R_EARTH, t.grid(), t.psi, t.h_obs, (100000.0, 0.0, 20000.0), D, 8) is None
    # the same direction towards the origin reaches the ground
    o = oracle.propagate_curved(cfg, -100000.0, 0.0, 20000.0, D[0], D[1], -D[2])
    assert o["status"][0] == -1
    # horizontal in the Cartesian frame at x = -50 km: 0.45 deg below the local
    # horizontal there, so it turns; at x = +50 km it moves outward
    o = oracle.propagate_curved(cfg, [-50000.0, 50000.0], 0.0, 9000.0, 1.0, 0.0, 0.0)
    assert list(o["status"]) == [oracle.DROP_NAMES.index("grazing"), oracle.DROP_NAMES.index("upward")]
    # straight up
    o = oracle.propagate_curved(cfg, 0.0, 0.0, 9000.0, 0.0, 0.0, -1.0)
    assert o["status"][0] == oracle.DROP_NAMES.index("upward")


def test_uniform_medium_straight_chord():
    alt = np.arange(0.0, 40001.0, 100.0)
    n = 1.0 + 2.5e-4
    t = oracle.build_tables(alt, np.full(alt.shape, n - 1.0), 1500.0, 50.0)
    cfg = oracle.Config(t, [0.0], [0.0], [10.0], earth_radius=R_EARTH)
    rng = np.random.default_rng(4)
    for _ in range(20):
        th, ph = math.radians(rng.uniform(0, 80)), rng.uniform(0, 2 * math.pi)
        D = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th)])
        P = np.array([rng.uniform(-2e4, 2e4), rng.uniform(-2e4, 2e4), rng.uniform(3000, 20000)])
        o = oracle.propagate_curved(cfg, P[0], P[1], P[2], D[0], D[1], -D[2])
        Q = P + np.array([0.0, 0.0, R_EARTH])
        r_obs = R_EARTH + 1500.0
        b = Q @ D
        c0 = Q @ Q - r_obs ** 2
        disc = b * b - c0
        if disc <= 0 or b >= 0:
            assert o["status"][0] >= 0
            continue
        s = -b - math.sqrt(disc)
        G = P + s * D
        assert o["status"][0] == -1
        assert abs(o["x_g"][0] - G[0]) < 1e-6 and abs(o["y_g"][0] - G[1]) < 1e-6
        assert abs(o["T"][0] - n * s / C_LIGHT) < 1e-9 * (n * s / C_LIGHT)
        assert abs(o["u_o"][0] - D[0]) < 1e-12 and abs(o["v_o"][0] - D[1]) < 1e-12


def test_radial_ray_is_the_vertical_flat_ray():
    t, cfg = _cfg()
    _, flat = _cfg(R=0.0)
    o = oracle.propagate_curved(cfg, 0.0, 0.0, 11234.5, 0.0, 0.0, 1.0)
    f = oracle.propagate(flat, 0.0, 0.0, 11234.5, 0.0, 0.0, 1.0)
    assert o["x_g"][0] == 0.0 and o["y_g"][0] == 0.0
    assert abs(o["T"][0] - f["T"][0]) < 1e-12 * f["T"][0]


def test_very_large_radius_is_the_plane_parallel_exact_path():
    # the curvature terms scale as 1/R (about 3e10 m^2 / R on a 100 km path):
    # at R = 1e16 m they are below 1e-5 m
    t, big = _cfg(R=1e16)
    _, flat = _cfg(R=0.0)
    rng = np.random.default_rng(8)
    m = 200
    th = np.radians(rng.uniform(0, 85, m))
    ph = rng.uniform(0, 2 * np.pi, m)
    u, v, w = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
    x, y, z = rng.uniform(-3000, 3000, m), rng.uniform(-3000, 3000, m), rng.uniform(2300, 30000, m)
    o = oracle.propagate_curved(big, x, y, z, u, v, w)
    e = oracle.propagate_exact(flat, x, y, z, u, v, w)
    assert np.all(o["status"] == -1)
    np.testing.assert_allclose(o["x_g"], e["x_g"], rtol=0, atol=2e-5)
    np.testing.assert_allclose(o["y_g"], e["y_g"], rtol=0, atol=2e-5)
    np.testing.assert_allclose(o["T"], e["T"], rtol=1e-9)
    np.testing.assert_allclose(o["u_o"], e["u_o"], rtol=0, atol=1e-9)


def test_run_switch():
    """Curved runs: every bunch traced exactly (no w_min cut); with a huge
    radius (1e16 m) the run equals the plane-parallel run with the exact
    grazing path."""
    atmo = synth.layered_atmosphere()
    segs = synth.shower_segments(5, 400, atmo, zenith_deg=70.0, xmax=400.0)
    tels = synth.telescopes_grid(n_side=5, pitch=150.0, radius=12.0)
    wl = synth.Workload("curved", atmo, tels, segs)
    r_big = oracle.run(oracle.Config.from_workload(wl, earth_radius=1e16), segs, nthreads=4)
    r_flat = oracle.run(oracle.Config.from_workload(wl, grazing_exact=True), segs, nthreads=4)
    assert r_big.n_bunches == r_flat.n_bunches and r_big.drops == r_flat.drops
    np.testing.assert_array_equal(r_big.offsets, r_flat.offsets)
    np.testing.assert_allclose(r_big.rec, r_flat.rec, rtol=1e-9, atol=2e-5)
    r = oracle.run(oracle.Config.from_workload(wl, earth_radius=R_EARTH), segs, nthreads=4)
    assert r.drops["grazing"] == 0 or r.drops["grazing"] < r.n_bunches // 100
    assert len(r.seg) > 0
    # the records are those of propagate_curved on each hit's bunch
    bd = oracle.bunch_details(oracle.Config.from_workload(wl, earth_radius=R_EARTH), segs, r.seg, r.k)
    np.testing.assert_array_equal(bd["status"], -1)
    np.testing.assert_array_equal(bd["x_g"] - tels.x[r.tel], r.rec[:, 0])
    np.testing.assert_array_equal(bd["h_e"], r.rec[:, 5])
    with pytest.raises(ValueError):
        oracle.profile(oracle.Config.from_workload(wl, earth_radius=R_EARTH), segs,
                       np.linspace(1000, 0, 100), 10.0)
