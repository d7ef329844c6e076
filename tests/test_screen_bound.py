"""The screening pass's per-step cull, checked on the oracle's bunches (CPU).

A step is left out of the soft response's screening when no sphere centre lies in
an annulus around G, the ground point of the step's axis: every bunch the FP64
pass keeps reaches the ground within [r_lo, r_hi] of G (the displacement of
App. B, taken through its four-term moment series, bounded by the range of psi),
and a bunch weights a sphere of cut radius R only if its ground point lies within
R / w_o of the centre.  This test restates the bound in numpy and checks it against the
oracle's ground points and soft weights on the 20 deg and 72 deg differentiation
showers and on a profile whose psi is not monotone; it also records how many
bunches the cull removes."""
import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import synth

W_MIN = 0.1          # grazing cut of the default parameters
Z_CUT = 40.0         # the soft weight is exactly zero below z = -40
SCREEN_MARGIN = 0.01


def annulus(dw, psi, sd):
    """Per step: valid, G, r_lo, r_hi, inner, outer (the bound as the screening
    pass evaluates it, margins included)."""
    s = dw.segs
    pmin, pmax = psi.min(), psi.max()
    falls = bool(np.all(np.diff(psi) <= 0))
    x0 = (pmax - pmin) / (1.0 + pmin)
    b0 = (0.5 if falls else 0.8) * x0
    rho2 = 1.0 if falls else (1.0 + pmax) / (1.0 + pmin)
    reff = np.sqrt(dw.tels.r ** 2 + 2 * dw.tels.r * dw.sigma * Z_CUT) * (1 + 1e-9) + SCREEN_MARGIN
    u, v, w = s.u, s.v, s.w
    ct, st = sd["cos_t"], sd["sin_t"]
    with np.errstate(invalid="ignore", divide="ignore"):
        sa = np.sqrt(np.maximum(0.0, (1 - w) * (1 + w)))
        s_hi = st * (1 + 1e-9) + 1e-12
        s_lo = np.maximum(st * (1 - 1e-9) - 1e-12, 0.0)
        wp_hi = np.minimum(1.0, w * ct + sa * s_hi + 1e-12)
        wp_lo = np.maximum(w * ct - sa * s_hi - 1e-12, W_MIN)
        iw2 = 1.0 / wp_lo ** 2
        B = b0 * iw2
        t_max = np.sqrt((1 - wp_lo) * (1 + wp_lo)) / wp_lo
        dh0 = s.h0 - dw.obs_level
        dh_top = np.maximum(dh0, 0.0)
        dh_bot = np.maximum(dh0 - s.length * w, 0.0)
        f_lo = s_lo / wp_hi - B * t_max
        f_hi = s_hi / (wp_lo * w) + B * t_max
        r_lo = np.where(f_lo > 0, dh_bot * f_lo, 0.0)
        r_hi = dh_top * f_hi
        wo2 = 1.0 - np.minimum(1.0, rho2 * (1 - wp_lo) * (1 + wp_lo))
        reach = reff.max() / np.sqrt(wo2)
        m = 0.1 + 1e-6 * (dh_top + r_hi)
        inner = np.maximum(r_lo - reach - m, 0.0)
        outer = r_hi + reach + m
        gx = s.x0 + dh0 * (u / w)
        gy = s.y0 + dh0 * (v / w)
    valid = ((np.abs(u * u + v * v + w * w - 1) <= 1e-9) & (w >= 0.05) & (sd["status"] < 0)
             & (x0 * iw2 <= 0.5) & (wo2 > 1e-6))
    return valid, gx, gy, r_lo, r_hi, inner, outer, falls


def cases():
    yield "20deg", synth.diff_showers(1, 3000), None
    yield "72deg", synth.diff_showers(1, 3000, zenith_deg=72.0), None
    dw = synth.diff_showers(1, 3000)
    th = dw.theta0.copy()
    th[:dw.n_knots] = 0.1 * (-1.0) ** np.arange(dw.n_knots)
    yield "non-monotone", dw, th


@pytest.mark.parametrize("name,dw,theta", list(cases()), ids=["20deg", "72deg", "non-monotone"])
def test_annulus_holds_every_weighted_bunch(name, dw, theta):
    spec = oracle.AtmoParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                                dw.top)
    t = oracle.tables_from_params(spec, dw.theta0 if theta is None else theta)
    psi = np.asarray(t.psi)
    cfg = oracle.Config(t, dw.tels.x, dw.tels.y, dw.tels.r, seed=dw.seed)
    sd = oracle.segment_details(cfg, dw.segs)
    nb = sd["n_b"].astype(np.int64)
    valid, gx, gy, r_lo, r_hi, inner, outer, falls = annulus(dw, psi, sd)
    assert falls == (theta is None)
    assert valid[sd["status"] < 0].mean() > 0.95
    # steps the cull removes: no sphere centre inside the annulus
    D2 = (gx[:, None] - dw.tels.x[None, :]) ** 2 + (gy[:, None] - dw.tels.y[None, :]) ** 2
    inside = (D2 >= inner[:, None] ** 2) & (D2 <= outer[:, None] ** 2)
    culled = valid & ~inside.any(axis=1)
    frac = nb[culled].sum() / nb.sum()
    # every bunch of a sample of the showers' bunches
    seg = np.repeat(np.arange(len(nb)), nb)
    k = np.arange(len(seg)) - np.repeat(np.cumsum(nb) - nb, nb)
    pick = np.random.default_rng(7).choice(len(seg), size=min(60000, len(seg)), replace=False)
    bd = oracle.bunch_details(cfg, dw.segs, seg[pick], k[pick])
    sp = seg[pick]
    kept = (bd["status"] < 0) & valid[sp]
    r = np.hypot(bd["x_g"] - gx[sp], bd["y_g"] - gy[sp])
    assert np.all(r[kept] >= r_lo[sp][kept]) and np.all(r[kept] <= r_hi[sp][kept])
    dx = bd["x_g"][:, None] - dw.tels.x[None, :]
    dy = bd["y_g"][:, None] - dw.tels.y[None, :]
    b = dx * bd["u_o"][:, None] + dy * bd["v_o"][:, None]
    z = (dw.tels.r[None, :] ** 2 - (dx * dx + dy * dy - b * b)) / (2.0 * dw.tels.r[None, :] * dw.sigma)
    weighted = (bd["status"] < 0)[:, None] & (z >= -Z_CUT)
    assert weighted.sum() > 50
    # each weighted (bunch, sphere) pair has its sphere centre inside its step's annulus
    wi, wk = np.nonzero(weighted & valid[sp][:, None])
    assert np.all(inside[sp[wi], wk])
    assert not culled[sp[weighted.any(axis=1)]].any()
    print(f"{name}: cull removes {frac:.3f} of the bunches ({culled.mean():.3f} of the steps)")
    assert frac > 0.2
