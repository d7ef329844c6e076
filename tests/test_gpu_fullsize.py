"""The three large workloads at their full sizes, in the launch configuration the
benchmark uses, checked where the oracle can follow: exact bunch counts for every
step (or every step of sampled showers), oracle records for sampled steps with
their original random numbers, and properties that hold at any size.

* hadron-like showers at 0, 20, 40 and 60 deg zenith, 5e7 steps each (2.5-4.3e9
  bunches), mixed precision, output streamed in chunks of 8 388 608 records (256 MB);
* 256 showers of 30 GeV - 30 TeV (~3e8 steps, ~1.6e10 bunches) in one persistent
  launch;
* differentiation workload, 64 showers x 5e5 steps: forward against the oracle on
  sampled steps, gradient against central differences of the forward along random
  directions."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth
from paper_2006_14927_amd.objective import telescope_loss

from gpu_helpers import compare_records, handles, params, say

pytestmark = pytest.mark.gpu


def _sampled_view(g_off, g_rec, g_ids, keep, n_groups):
    """Records of the kept steps, regrouped into CSR over the same groups."""
    counts = np.diff(g_off)
    group = np.repeat(np.arange(len(counts)), counts)[keep]
    off = np.zeros(n_groups + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(group, minlength=n_groups))
    return dict(offsets=off, rec=g_rec[keep], ids=g_ids[keep])


@pytest.mark.parametrize("zenith", [0.0, 20.0, 40.0, 60.0])
def test_hadron_like_full_size_streamed(zenith):
    import torch
    wl = synth.hadron_like(zenith)
    assert wl.segs.n == 50_000_000 and wl.segs.n_showers == 1
    cfg = oracle.Config.from_workload(wl)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    st = ckv.Streamer(d, atmo, tels, params(wl, ckv.CKV_MIXED))
    say(f"[gpu] hadron {zenith} deg full: {st.total_bunches} bunches")
    # exact bunch counts of every step against the oracle, in slices
    n_b_gpu = ckv.count(d, atmo, params(wl, ckv.CKV_MIXED)).cpu().numpy()
    total = 0
    for a in range(0, wl.segs.n, 5_000_000):
        idx = np.arange(a, min(a + 5_000_000, wl.segs.n))
        nb = oracle.segment_details(cfg, wl.segs.take(idx))["n_b"].astype(np.int64)
        np.testing.assert_array_equal(n_b_gpu[idx], nb)
        total += int(nb.sum())
    assert total == st.total_bunches > 2_000_000_000
    # stream the output; keep the records of every 997th step
    idx = np.arange(0, wl.segs.n, 997)
    idx_t = torch.as_tensor(idx, device="cuda")
    n_tel = tels.n
    parts, n_chunks, agg, end = [], 0, dict(n_bunches=0, n_hits=0), 0
    for ch in st.chunks():
        res = ch.result
        assert res["error"] == 0 and ch.begin == end     # chunks tile the steps
        end = ch.end
        assert 0 < res["n_records"] <= st.capacity
        agg["n_bunches"] += st.bunches(ch.begin, ch.end)
        agg["n_hits"] += res["n_records"]
        n_chunks += 1
        off = ch.tel_offsets.cpu().numpy()
        ids = ch.ids.clone()
        ids[:, 0] += ch.begin            # ids count steps from the start of the chunk's range
        keep = torch.isin(ids[:, 0], idx_t).cpu().numpy()
        parts.append(_sampled_view(off, ch.records.cpu().numpy(), ids.cpu().numpy(), keep, n_tel))
    say(f"[gpu] streamed {n_chunks} chunks ({st.n_resumed} resumed, {st.n_reruns} rerun), "
        f"{agg['n_hits']} records")
    assert end == wl.segs.n and agg["n_bunches"] == st.total_bunches and n_chunks >= 2
    # per telescope, consecutive chunks concatenate in (step, bunch) order
    off = np.zeros(n_tel + 1, dtype=np.int64)
    off[1:] = np.cumsum(sum(np.diff(p["offsets"]) for p in parts))
    rec = np.concatenate([p["rec"][p["offsets"][t]:p["offsets"][t + 1]]
                          for t in range(n_tel) for p in parts])
    ids = np.concatenate([p["ids"][p["offsets"][t]:p["offsets"][t + 1]]
                          for t in range(n_tel) for p in parts])
    sub = wl.segs.take(idx)
    ores = oracle.run(cfg, sub, nthreads=16, seg_id=idx)
    rep = compare_records(wl, cfg, ores, dict(offsets=off, rec=rec, ids=ids), ckv.CKV_MIXED,
                          segs=sub, seg_map=idx)
    say(f"[gpu] hadron {zenith} deg full, sampled steps: {rep}")


def test_batched_256_showers_full_size():
    import torch
    wl = synth.batched_showers(256)
    sizes = np.diff(wl.segs.seg_offsets)
    say(f"[gpu] batched full: {wl.segs.n} steps, showers {sizes.min()}..{sizes.max()}")
    assert wl.segs.n > 2e8
    cfg = oracle.Config.from_workload(wl)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED)
    n_b = ckv.count(d, atmo, p)
    total = int(n_b.sum())
    cap = int(0.02 * total)
    r = ckv.Runner(d, atmo, tels, p, cap)
    out = r.run()
    torch.cuda.synchronize()
    res = out.result()
    if res["overflow"]:
        cap = int(res["n_hits"]) + 1024
        say(f"[gpu] rerun with capacity {cap}")
        del r, out
        r = ckv.Runner(d, atmo, tels, p, cap)
        out = r.run()
        torch.cuda.synchronize()
        res = out.result()
    assert res["overflow"] == 0 and res["error"] == 0 and res["n_bunches"] == total
    say(f"[gpu] batched full: {total} bunches, {res['n_hits']} records, {res['n_tiles']} tiles")
    n_b = n_b.cpu().numpy()
    off = out.tel_offsets.cpu().numpy()
    n_tel = tels.n
    for s in range(0, 256, 16):
        lo, hi = int(wl.segs.seg_offsets[s]), int(wl.segs.seg_offsets[s + 1])
        one = wl.segs.take_shower(s, np.arange(hi - lo))
        nb = oracle.segment_details(cfg, one)["n_b"].astype(np.int64)
        np.testing.assert_array_equal(n_b[lo:hi], nb)
        # sampled steps of this shower
        loc = np.arange(0, hi - lo, 97)
        sub = wl.segs.take_shower(s, loc)
        ores = oracle.run(cfg, sub, nthreads=16, seg_id=loc)
        a, b = int(off[s * n_tel]), int(off[(s + 1) * n_tel])
        ids = out.ids[a:b].cpu().numpy()
        ids[:, 0] -= lo                  # index in the step arrays -> index in the shower
        keep = np.isin(ids[:, 0], loc)
        g = _sampled_view(off[s * n_tel:(s + 1) * n_tel + 1] - a, out.records[a:b].cpu().numpy(),
                          ids, keep, n_tel)
        rep = compare_records(wl, cfg, ores, g, ckv.CKV_MIXED, segs=sub, seg_map=loc)
        if s % 64 == 0:
            say(f"[gpu] batched full, shower {s}: {rep}")


def test_differentiation_full_size():
    import torch
    dw = synth.diff_showers()
    assert dw.segs.n == 32_000_000 and dw.segs.n_showers == 64
    spec = ckv.ParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level, dw.step,
                         dw.top)
    model = ckv.SoftModel(dw.segs, dw.tels, spec, dw.theta0, dw.sigma, seed=dw.seed)
    St, At = model.forward(dw.theta_target)
    # forward against the oracle on 20 000 consecutive steps of shower 5 (their own
    # random numbers: step indices from 240 000), at the start and target parameters
    o_spec = oracle.AtmoParamSpec(dw.eta0, dw.layer_bounds, dw.n_knots, dw.knot_top, dw.obs_level,
                                  dw.step, dw.top)
    a0, m = 240_000, 20_000
    base = int(dw.segs.seg_offsets[5])
    sub = dw.segs.take_shower(5, np.arange(a0, a0 + m))
    part = ckv.SoftModel(model.dsegs.view(base + a0, base + a0 + m), dw.tels, spec, dw.theta0,
                         dw.sigma, seed=dw.seed)
    c0 = oracle.Config(oracle.tables_from_params(o_spec, dw.theta0), dw.tels.x, dw.tels.y, dw.tels.r,
                       seed=dw.seed)
    nb = oracle.segment_details(c0, sub)["n_b"].astype(np.int64)
    np.testing.assert_array_equal(part.n_b.cpu().numpy(), nb)
    for th in (dw.theta0, dw.theta_target):
        c = oracle.Config(oracle.tables_from_params(o_spec, th), dw.tels.x, dw.tels.y, dw.tels.r,
                          seed=dw.seed)
        So, Ao = oracle.soft(c, sub, nb, dw.sigma, nthreads=16, seg_id_base=[a0])
        Sg, Ag = part.forward(th)
        torch.cuda.synchronize()
        assert So.sum() > 0
        np.testing.assert_allclose(Sg.cpu().numpy(), So, rtol=1e-10, atol=1e-12 * So.max())
        np.testing.assert_allclose(Ag.cpu().numpy(), Ao, rtol=1e-10, atol=1e-12 * np.abs(Ao).max())
        say(f"[gpu] diff full: soft response on {m} steps of shower 5 matches (S sum {So.sum():.6e})")
    del part
    # gradient . v against central differences of the forward, full size
    theta = torch.tensor(dw.theta0, dtype=torch.float64, requires_grad=True)
    S, A = ckv.soft_response(theta, model)
    telescope_loss(S, A, St, At).backward()
    g = theta.grad.numpy()
    assert np.isfinite(g).all()
    rng = np.random.default_rng(11)
    scale = np.concatenate([np.full(dw.n_knots, 1.0), dw.theta0[dw.n_knots:]])
    for _ in range(2):
        v = rng.normal(size=g.shape) * scale

        def L_at(th):
            S_, A_ = model.forward(th)
            return float(telescope_loss(S_, A_, St, At))

        def central(hh):
            return (L_at(dw.theta0 + hh * v) - L_at(dw.theta0 - hh * v)) / (2 * hh)

        fd = (4.0 * central(1e-4) - central(2e-4)) / 3.0
        say(f"[gpu] diff full: g.v={g @ v:.10e} fd={fd:.10e}")
        assert g @ v == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g * v).sum())
