"""Differentiation: the soft telescope response and its gradient with respect to
the atmosphere parameters (64 log(n-1) knots + 8 layer scale heights), through
torch.autograd, against FP64 central finite differences of the oracle."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth
from paper_2006_14927_amd.objective import telescope_loss

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def np_loss(S, A, St, At):
    use = (St >= 100.0) & (S > 0)
    rel = (S - St) / (St + 10.0)
    M = A / np.where(use, S, 1.0)
    Mt = At / np.where(use, St, 1.0)
    return float(np.sum(rel * rel) + np.sum(np.where(use, M - Mt, 0.0) ** 2))


class Oracle:
    def __init__(self, dw):
        self.dw = dw
        self.spec = oracle.AtmoParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top,
                                         dw.obs_level, dw.step, dw.top)
        cfg0 = self.cfg(dw.theta0)
        self.nb = oracle.segment_details(cfg0, dw.segs)["n_b"].astype(np.int64)

    def cfg(self, theta):
        t = oracle.tables_from_params(self.spec, theta)
        return oracle.Config(t, self.dw.tels.x, self.dw.tels.y, self.dw.tels.r, seed=self.dw.seed)

    def SA(self, theta):
        return oracle.soft(self.cfg(theta), self.dw.segs, self.nb, self.dw.sigma, nthreads=16)


def gpu_model(dw):
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    return ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed)


@pytest.fixture(scope="module")
def small():
    dw = synth.diff_showers(2, 5000)
    return dw, Oracle(dw), gpu_model(dw)


def test_parameterised_tables_and_frozen_counts(small):
    dw, orc, model = small
    psi, P = model.atmo0.tables()
    t = oracle.tables_from_params(orc.spec, dw.theta0)
    np.testing.assert_array_equal(psi, t.psi)
    np.testing.assert_allclose(P, t.P, rtol=1e-13, atol=0)
    np.testing.assert_array_equal(model.n_b.cpu().numpy(), orc.nb)


def bumpy_theta(dw):
    """theta0 with knots alternating +-0.1: psi rises with altitude at hundreds of
    nodes, so the screening cull takes its bound for profiles that are not monotone."""
    th = dw.theta0.copy()
    th[:dw.n_knots] = 0.1 * (-1.0) ** np.arange(dw.n_knots)
    return th


@pytest.mark.parametrize("which", ["theta0", "target", "bumpy"])
def test_soft_forward_matches_oracle(small, which):
    """The listed forward (screening pass with its per-step cull, then FP64 over the
    list) gives the oracle's S and A, also on a profile that is not monotone."""
    import torch
    dw, orc, model = small
    th = {"theta0": dw.theta0, "target": dw.theta_target, "bumpy": bumpy_theta(dw)}[which]
    if which == "bumpy":
        assert (np.diff(oracle.tables_from_params(orc.spec, th).psi) > 0).sum() > 100
    S, A = model.forward(th)
    torch.cuda.synchronize()
    So, Ao = orc.SA(th)
    assert So.sum() > 1e3 and (So > 100).sum() >= 4
    np.testing.assert_allclose(S.cpu().numpy(), So, rtol=1e-10, atol=1e-12 * So.max())
    np.testing.assert_allclose(A.cpu().numpy(), Ao, rtol=1e-10, atol=1e-12 * np.abs(Ao).max())


@pytest.mark.parametrize("n_tel", [1, 37])
def test_soft_forward_with_odd_sphere_counts(n_tel):
    """The screening cull splits the sphere table between the two half-waves
    ([0, nh) and [n - nh, n), one sphere tested twice when n is odd): the listed
    forward still gives the oracle's S and A with 1 and 37 spheres."""
    import dataclasses
    import torch
    dw = synth.diff_showers(2, 5000)
    t = synth.telescopes_disk(n=n_tel, disk_radius=300.0, seed=11)
    dw = dataclasses.replace(dw, tels=t)
    orc = Oracle(dw)
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    # a list that holds every bunch, so that the forward takes the listed path
    model = ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed,
                          list_capacity=int(orc.nb.sum()))
    S, A = model.forward(dw.theta0)
    torch.cuda.synchronize()
    n, cap = model.list_state()
    assert 0 < n <= cap
    So, Ao = orc.SA(dw.theta0)
    assert So.sum() > 100
    np.testing.assert_allclose(S.cpu().numpy(), So, rtol=1e-10, atol=1e-12 * So.max())
    np.testing.assert_allclose(A.cpu().numpy(), Ao, rtol=1e-10, atol=1e-12 * np.abs(Ao).max())


@pytest.mark.parametrize("which", ["theta0", "bumpy"])
def test_unlisted_forward_matches_oracle(small, which):
    """Without a list the FP64 tile forward computes S and A from every bunch of
    the steps the cull keeps: the oracle's S and A, also on a profile that is not
    monotone."""
    import torch
    dw, orc, _ = small
    th = dw.theta0 if which == "theta0" else bumpy_theta(dw)
    model = gpu_model_nolist(dw)
    S, A = model.forward(th)
    torch.cuda.synchronize()
    So, Ao = orc.SA(th)
    np.testing.assert_allclose(S.cpu().numpy(), So, rtol=1e-10, atol=1e-12 * So.max())
    np.testing.assert_allclose(A.cpu().numpy(), Ao, rtol=1e-10, atol=1e-12 * np.abs(Ao).max())


def test_gradient_matches_oracle_finite_differences(small):
    """All 72 coordinates: Richardson-extrapolated central differences of the
    FP64 oracle loss, (4 D(h) - D(2h)) / 3 (plain central differences at
    h = 1e-4 still carry ~1e-4 relative truncation error here)."""
    import torch
    dw, orc, model = small
    St_o, At_o = orc.SA(dw.theta_target)
    St, At = model.forward(dw.theta_target)
    theta = torch.tensor(dw.theta0, dtype=torch.float64, requires_grad=True)
    S, A = ckv.soft_response(theta, model)
    L = telescope_loss(S, A, St, At)
    L.backward()
    g = theta.grad.numpy().copy()
    assert np.isfinite(g).all()
    L_o0 = np_loss(*orc.SA(dw.theta0), St_o, At_o)
    assert float(L.detach()) == pytest.approx(L_o0, rel=1e-9)

    def central(j, step):
        tp, tm = dw.theta0.copy(), dw.theta0.copy()
        tp[j] += step
        tm[j] -= step
        return (np_loss(*orc.SA(tp), St_o, At_o) - np_loss(*orc.SA(tm), St_o, At_o)) / (2 * step)

    fd = np.zeros_like(g)
    for j in range(len(g)):
        step = 1e-4 if j < dw.n_knots else 1e-4 * dw.theta0[j]
        fd[j] = (4.0 * central(j, step) - central(j, 2 * step)) / 3.0
    floor = 1e-3 * np.abs(fd).max()
    err = np.abs(g - fd) / np.maximum(np.abs(fd), floor)
    say(f"[gpu] grad vs oracle FD: max rel err {err.max():.2e} (|g|max {np.abs(g).max():.3e})")
    assert np.abs(fd).max() > 0
    assert err.max() <= 1e-5, (np.argsort(-err)[:5], err[np.argsort(-err)[:5]])


def test_directional_derivative_larger_instance():
    """8 showers x 2e4 steps: gradient . v against central differences of the
    FP64 response along 4 random directions v."""
    import torch
    dw = synth.diff_showers(8, 20000)
    model = gpu_model(dw)
    St, At = model.forward(dw.theta_target)
    theta = torch.tensor(dw.theta0, dtype=torch.float64, requires_grad=True)
    S, A = ckv.soft_response(theta, model)
    telescope_loss(S, A, St, At).backward()
    g = theta.grad.numpy()
    rng = np.random.default_rng(7)
    scale = np.concatenate([np.full(dw.n_knots, 1.0), dw.theta0[dw.n_knots:]])
    for _ in range(4):
        v = rng.normal(size=g.shape) * scale
        h = 1e-4

        def L_at(th):
            S_, A_ = model.forward(th)
            return float(telescope_loss(S_, A_, St, At))

        def central(hh):
            return (L_at(dw.theta0 + hh * v) - L_at(dw.theta0 - hh * v)) / (2 * hh)

        fd = (4.0 * central(h) - central(2 * h)) / 3.0
        say(f"[gpu] directional: g.v={g @ v:.10e} fd={fd:.10e}")
        assert g @ v == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g * v).sum())


def _tables_backward(model, theta, gS, gA):
    import torch
    g_psi, g_P = model.backward_tables(theta, gS, gA)
    torch.cuda.synchronize()
    return g_psi.cpu().numpy().copy(), g_P.cpu().numpy().copy()


def _random_cotangents(model, seed):
    import torch
    rng = np.random.default_rng(seed)
    gS = torch.tensor(rng.normal(size=model.shape), dtype=torch.float64, device="cuda")
    gA = torch.tensor(rng.normal(size=model.shape) * 1e-3, dtype=torch.float64, device="cuda")
    return gS, gA


def _assert_same_gradient(a, b):
    for x, y in zip(a, b):
        scale = np.abs(y).max()
        assert scale > 0
        np.testing.assert_allclose(x, y, rtol=1e-11, atol=1e-13 * scale)


def test_listed_adjoint_equals_full_recompute(small):
    """The adjoint over the forward's list of weighted bunches gives the gradient
    of the adjoint that recomputes every bunch (FP64 sums in another order)."""
    dw, orc, model = small
    full = gpu_model_nolist(dw)
    model.forward(dw.theta0)
    full.forward(dw.theta0)
    n, cap = model.list_state()
    nb = int(model.n_b.sum())
    say(f"[gpu] soft list: {n} of {nb} bunches ({n / nb:.3%}), capacity {cap}")
    assert 0 < n <= cap
    gS, gA = _random_cotangents(model, 11)
    _assert_same_gradient(_tables_backward(model, dw.theta0, gS, gA),
                          _tables_backward(full, dw.theta0, gS, gA))


def gpu_model_nolist(dw, **kw):
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    return ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed, use_list=False,
                         **kw)


@pytest.fixture(scope="module")
def inclined():
    dw = synth.diff_showers(2, 5000, zenith_deg=72.0)
    return dw, Oracle(dw), gpu_model(dw)


@pytest.mark.parametrize("which", ["small", "inclined"])
def test_list_holds_every_weighted_bunch(which, request):
    """The forward's list (the mixed screening pass against spheres of the cut
    radius plus 1 cm, plus every bunch whose ground-error bound passes half that
    margin) names every bunch of the oracle with z >= -40 at some sphere, each
    once; the others it names lie just outside the cut or carry a large bound.
    Also at 72 deg zenith, where w ~ 0.3 magnifies the mixed path's errors."""
    import torch
    dw, orc, model = request.getfixturevalue(which)
    model.forward(dw.theta0)
    n, cap = model.list_state()
    assert n <= cap
    ids = model.list_ids[:n].cpu().numpy().view(np.uint64)
    seg = (ids >> np.uint64(24)).astype(np.int64)
    k = (ids & np.uint64((1 << 24) - 1)).astype(np.int64)
    key = seg * (1 << 24) + k
    assert len(np.unique(key)) == n
    cfg = orc.cfg(dw.theta0)
    nb = orc.nb
    all_seg = np.repeat(np.arange(len(nb)), nb)
    all_k = np.arange(len(all_seg)) - np.repeat(np.cumsum(nb) - nb, nb)
    zmax = np.full(len(all_seg), -np.inf)
    tx, ty, tr = dw.tels.x, dw.tels.y, dw.tels.r
    for lo in range(0, len(all_seg), 50000):
        sl = slice(lo, lo + 50000)
        bd = oracle.bunch_details(cfg, dw.segs, all_seg[sl], all_k[sl])
        ok = bd["status"] < 0
        dx = bd["x_g"][:, None] - tx[None, :]
        dy = bd["y_g"][:, None] - ty[None, :]
        b = dx * bd["u_o"][:, None] + dy * bd["v_o"][:, None]
        z = (tr[None, :] ** 2 - (dx * dx + dy * dy - b * b)) / (2.0 * tr[None, :] * dw.sigma)
        zmax[sl] = np.where(ok, z.max(axis=1), -np.inf)
    want = zmax >= -40.0
    okey = all_seg * (1 << 24) + all_k
    listed = np.isin(okey, key)
    assert not np.isin(key, okey, invert=True).any()
    assert np.all(listed[want]), (~listed[want]).sum()
    assert want.sum() > 100
    extra = listed & ~want
    # the rest lie just outside the cut, or were listed for their error bound
    bd = oracle.bunch_details(cfg, dw.segs, all_seg[extra], all_k[extra])
    winv = 1.0 / bd["w"]
    bound = (bd["h_e"] - dw.obs_level) * winv * (1e-8 * (1.0 + winv) + 5e-10 * winv * winv)
    near = zmax[extra] > -40.5
    assert np.all(near | (bound > 0.004)), np.sort(zmax[extra][~near])[:5]
    say(f"[gpu] soft list ({dw.name}): {n} ids, {want.sum()} weighted bunches of the oracle, "
        f"{near.sum()} candidates just outside the cut, {(~near).sum()} listed for their bound")


def test_list_overflow_recomputes_everything_then_grows(small):
    """A list too small for the forward is incomplete: the adjoint recomputes every
    bunch (same gradient); grow_list enlarges it and the next pass uses it."""
    dw, orc, model = small
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    m = ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed, list_capacity=16)
    full = gpu_model_nolist(dw)
    gS, gA = _random_cotangents(m, 12)
    S16, A16 = m.forward(dw.theta0)
    S, A = full.forward(dw.theta0)
    n, cap = m.list_state()
    assert cap == 16 and n > cap
    # the incomplete list falls back to the FP64 tile forward over every bunch
    S16, A16, S, A = (x.cpu().numpy() for x in (S16, A16, S, A))
    assert S.sum() > 1e3
    np.testing.assert_allclose(S16, S, rtol=1e-12, atol=1e-12 * S.max())
    np.testing.assert_allclose(A16, A, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    ref = _tables_backward(full, dw.theta0, gS, gA)
    _assert_same_gradient(_tables_backward(m, dw.theta0, gS, gA), ref)
    assert m.grow_list()
    m.forward(dw.theta0)
    n2, cap2 = m.list_state()
    assert n2 == n and cap2 > n       # the screening list does not depend on the capacity
    _assert_same_gradient(_tables_backward(m, dw.theta0, gS, gA), ref)
    assert not m.grow_list()


def test_soft_list_argument_validation(small):
    """A list with negative capacity, no count or no ids (capacity > 0) is refused
    on the host by both entry points, before any work is queued."""
    import ctypes as C
    dw, orc, model = small
    L = ckv.lib()
    atmo = model._atmo(dw.theta0)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    ws = (ptr(model.workspace), model.workspace.numel())
    S = model.g_psi.new_empty(model.shape)
    for bad in (ckv._SoftList(model.list_ids.data_ptr(), -1, model.list_count.data_ptr()),
                ckv._SoftList(model.list_ids.data_ptr(), 10, None),
                ckv._SoftList(None, 10, model.list_count.data_ptr())):
        rc = L.ckv_soft_forward(C.byref(model._segs), C.byref(model._showers), C.byref(model.params),
                                atmo.handle, model.tels.handle, ptr(model.n_b), ptr(S), ptr(S),
                                C.byref(bad), None, *ws, None)
        assert rc == -1 and b"soft list" in L.ckv_last_error()
        rc = L.ckv_soft_backward(C.byref(model._segs), C.byref(model._showers), C.byref(model.params),
                                 atmo.handle, model.tels.handle, ptr(model.n_b), ptr(S), ptr(S),
                                 ptr(model.g_psi), ptr(model.g_P), C.byref(bad), None, *ws, None)
        assert rc == -1 and b"soft list" in L.ckv_last_error()


def test_listed_adjoint_skips_ids_that_name_no_bunch(small):
    """Ids past the last step, or past a step's bunch count, are skipped by the
    listed adjoint: appended to a real list they leave the gradient unchanged."""
    import torch
    dw, orc, model = small
    model.forward(dw.theta0)
    gS, gA = _random_cotangents(model, 13)
    ref = _tables_backward(model, dw.theta0, gS, gA)
    n, cap = model.list_state()
    assert n + 3 <= cap
    nb = model.n_b.cpu().numpy()
    step = int(np.flatnonzero(nb > 0)[0])
    bogus = np.array([(dw.segs.n + 5) << 24, (step << 24) | int(nb[step] + 3), 2 ** 63 - 1],
                     dtype=np.int64)
    model.list_ids[n:n + 3] = torch.from_numpy(bogus).to(model.list_ids.device)
    model.list_count.fill_(n + 3)
    torch.cuda.synchronize()
    _assert_same_gradient(_tables_backward(model, dw.theta0, gS, gA), ref)


def _bad_offsets_model(dw, offsets):
    """A model whose device shower offsets are replaced after construction."""
    import torch
    m = gpu_model_nolist(dw)
    m.dsegs.seg_offsets.copy_(torch.as_tensor(np.asarray(offsets, dtype=np.int64)))
    torch.cuda.synchronize()
    return m


def test_soft_entry_points_report_bad_offsets(small):
    """Shower offsets that do not end at the step count are caught on the device
    (init kernel): nothing is computed and both entry points report error bit 0,
    which SoftModel turns into an exception."""
    dw, orc, model = small
    n = dw.segs.n
    for use_list in (False, True):
        m = _bad_offsets_model(dw, [0, n // 2, n - 7])
        m.use_list = use_list
        if use_list:
            m._alloc_list(1 << 16)
        with pytest.raises(ckv.CkvError, match="error flags 1"):
            m.forward(dw.theta0)
        gS, gA = _random_cotangents(m, 3)
        with pytest.raises(ckv.CkvError, match="error flags 1"):
            m.backward_tables(dw.theta0, gS, gA)


def test_soft_entry_points_report_oversized_tile(small):
    """A frozen count that puts 2^30 bunches or more into one 32-step tile is
    refused by every soft kernel's tile guard (the tile is left out) and
    reported as error bit 1, with or without the screening list."""
    import torch
    dw, orc, model = small
    for use_list in (False, True):
        m = gpu_model_nolist(dw) if not use_list else gpu_model(dw)
        nb = m.n_b.clone()
        step = int(torch.nonzero(nb > 0)[0])
        m.n_b[step] = 1 << 31
        torch.cuda.synchronize()
        with pytest.raises(ckv.CkvError, match="error flags 2"):
            m.forward(dw.theta0)
        m.n_b.copy_(nb)
        torch.cuda.synchronize()
        S, A = m.forward(dw.theta0)
        assert float(S.sum()) > 0
