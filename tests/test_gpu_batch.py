"""Batching: many showers of uneven size in one persistent launch, the whole run
captured into a HIP graph, and the launch-shape autotuner."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import autotune, ckv, synth

from gpu_helpers import compare_records, gpu_run, handles, params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batched():
    # 256 showers, 30 GeV..30 TeV, step counts scaled by 5e-4 (5 .. 2000 steps each)
    wl = synth.batched_showers(256, seg_scale=5e-4)
    cfg = oracle.Config.from_workload(wl)
    return wl, cfg, oracle.run(cfg, wl.segs, nthreads=8)


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_batched_showers_parity(batched, precision):
    wl, cfg, r = batched
    sizes = np.diff(wl.segs.seg_offsets)
    assert wl.segs.n_showers == 256 and sizes.min() < 32 < sizes.max()
    g = gpu_run(wl, precision)
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    say(f"[gpu] batched prec={precision}: tiles={res['n_tiles']} {rep}")


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_more_showers_than_the_scatter_stages(precision):
    """2100 showers of 1..160 steps: more than the 2048 whose tile bounds the scatter
    keeps in LDS, so it finds each record's shower in HBM; offsets, ids and records
    are still the oracle's."""
    wl = synth.batched_showers(2100, seg_scale=4e-5)
    assert wl.segs.n_showers == 2100
    cfg = oracle.Config.from_workload(wl)
    r = oracle.run(cfg, wl.segs, nthreads=8)
    g = gpu_run(wl, precision)
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    assert rep["matched"] > 40_000
    say(f"[gpu] 2100 showers prec={precision}: {rep}")


def test_graph_replays_match_eager(batched):
    import torch
    wl, cfg, r = batched
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED)
    cap = len(r.seg) + 4096
    eager = ckv.Runner(d, atmo, tels, p, cap)
    out = eager.run()
    torch.cuda.synchronize()
    n = out.result()["n_records"]
    ref = (out.tel_offsets.cpu().clone(), out.records[:n].cpu().clone(), out.ids[:n].cpu().clone())
    gr = ckv.GraphRunner(ckv.Runner(d, atmo, tels, p, cap))
    other = ckv.Runner(ckv.DeviceSegments(synth.vertical_gamma(3000).segs), atmo, tels, p, 100000)
    for rep in range(4):
        o = gr.runner
        o.records.fill_(float("nan"))
        o.tel_offsets.fill_(-1)
        o.result_raw.zero_()
        other.run()                       # eager work on the same device between replays
        torch.cuda.synchronize()
        go = gr.replay()
        torch.cuda.synchronize()
        res = go.result()
        assert res["n_records"] == n and res["overflow"] == 0
        assert torch.equal(go.tel_offsets.cpu(), ref[0])
        assert torch.equal(go.records[:n].cpu().view(torch.int32), ref[1].view(torch.int32))
        assert torch.equal(go.ids[:n].cpu(), ref[2])
        say(f"[gpu] graph replay {rep} ok")


def test_autotune_candidates_identical_and_cached(tmp_path, monkeypatch):
    import torch
    monkeypatch.setattr(autotune, "CACHE_PATH", str(tmp_path / "tune.json"))
    wl = synth.vertical_gamma()
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED)
    cands = [(16, 16), (32, 8), (64, 4), (32, 16)]
    entry = autotune.tune(d, atmo, tels, p, 200000, candidates=cands, reps=2)
    assert (entry["tile_segments"], entry["waves_per_group"]) in cands
    assert len(entry["table"]) == len(cands)
    again = autotune.tune(d, atmo, tels, p, 200000, candidates=cands, reps=2)
    assert again == entry                                   # served from the cache
    outs = []
    for ts, wv in cands:
        q = autotune.apply(p, {"tile_segments": ts, "waves_per_group": wv})
        o = ckv.Runner(d, atmo, tels, q, 200000).run()
        torch.cuda.synchronize()
        n = o.result()["n_records"]
        outs.append((o.tel_offsets.cpu().numpy(), o.records[:n].cpu().numpy().view(np.uint32)))
    for off, rec in outs[1:]:
        np.testing.assert_array_equal(off, outs[0][0])
        np.testing.assert_array_equal(rec, outs[0][1])


@pytest.mark.parametrize("mode", ["device", "host"])
def test_streamed_chunks_equal_one_shot(batched, mode):
    """Small output chunks force many ranges, some of them inside one shower and
    some spanning several; per (shower, telescope) the chunks concatenate to the
    one-shot output, bit for bit (ids shifted by each range's first step)."""
    import torch
    wl, cfg, r = batched
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED)
    one = gpu_run(wl, ckv.CKV_MIXED, handles_=(atmo, tels))
    n_tel, n_sh = tels.n, wl.segs.n_showers
    st = ckv.Streamer(d, atmo, tels, p, chunk_records=max(1000, len(r.seg) // 12), first_ratio=0.002,
                      plan_block=64)
    got = [[] for _ in range(n_sh * n_tel)]
    n_chunks = [0]

    def take(ch):
        n_chunks[0] += 1
        off = np.asarray(ch.tel_offsets.cpu() if mode == "device" else ch.tel_offsets)
        rec = (ch.records.cpu() if mode == "device" else ch.records).numpy().copy()
        ids = (ch.ids.cpu() if mode == "device" else ch.ids).numpy().copy()
        ids[:, 0] += ch.begin
        for loc in range(ch.shower_end - ch.shower_begin):
            for t in range(n_tel):
                gi = loc * n_tel + t
                got[(ch.shower_begin + loc) * n_tel + t].append(
                    (rec[off[gi]:off[gi + 1]], ids[off[gi]:off[gi + 1]]))

    if mode == "device":
        for ch in st.chunks():
            take(ch)
    else:
        st.to_host(take)
    torch.cuda.synchronize()
    say(f"[gpu] streamed ({mode}): {n_chunks[0]} chunks, {st.n_resumed} resumed, {st.n_reruns} rerun")
    assert n_chunks[0] >= 8
    o = one["offsets"]
    for gi in range(n_sh * n_tel):
        rec = np.concatenate([x[0] for x in got[gi]]) if got[gi] else np.zeros((0, 8), np.float32)
        ids = np.concatenate([x[1] for x in got[gi]]) if got[gi] else np.zeros((0, 2), np.int64)
        np.testing.assert_array_equal(rec.view(np.uint32), one["rec"][o[gi]:o[gi + 1]].view(np.uint32))
        np.testing.assert_array_equal(ids, one["ids"][o[gi]:o[gi + 1]])
