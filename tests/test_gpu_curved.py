"""Curved atmosphere (spherical shells of the Earth's radius; every bunch traced
exactly in FP64 with Bouguer's invariant) on the GPU, against the oracle's
curved variant (itself pinned against a brute-force shell tracer): bunch counts
and every drop counter bit-exact, hit sets and records to the FP64 tolerance
(both precisions trace these bunches in FP64); inclined showers at 70 and 84
degrees, where the light is emitted 10-280 km away, and a vertical one."""

import numpy as np
import pytest

import oracle
from paper_2006_14927_amd import ckv, synth

from gpu_helpers import F32, compare_records, gpu_run, handles, params, say

pytestmark = pytest.mark.gpu

R_EARTH = 6.371e6


@pytest.fixture(scope="module", params=[(70.0, 20000), (84.0, 60000), (0.0, 4000)],
                ids=["70deg", "84deg", "vertical"])
def shower(request):
    zen, n = request.param
    wl = synth.inclined(zen, n)
    cfg = oracle.Config.from_workload(wl, earth_radius=R_EARTH)
    return wl, cfg, oracle.run(cfg, wl.segs, nthreads=16)


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_curved_showers(shower, precision):
    wl, cfg, r = shower
    g = gpu_run(wl, precision, earth_radius=R_EARTH, capacity=4 * len(r.seg) + 4096)
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0, res
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops, (res, r.drops)
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    say(f"[gpu] curved {wl.name} prec={precision}: bunches={res['n_bunches']} "
        f"hits={res['n_hits']} drops={res['drops']} {rep}")


def test_curved_bunch_counts(shower):
    """ckv_count with the curved midpoint altitude, bit-exact against the oracle."""
    import torch
    wl, cfg, r = shower
    atmo, _ = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    nb = ckv.count(d, atmo, params(wl, ckv.CKV_MIXED, earth_radius=R_EARTH))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(nb.cpu().numpy(), r.n_b)


def test_very_large_radius_matches_the_flat_exact_path():
    """R = 1e16 m: the curved kernel reproduces the plane-parallel run with the
    exact grazing path (curvature terms ~1e-6 m at this radius)."""
    wl = synth.inclined(70.0, 8000)
    a = gpu_run(wl, ckv.CKV_FP64, earth_radius=1e16)
    b = gpu_run(wl, ckv.CKV_FP64, grazing_exact=True)
    assert a["result"]["n_bunches"] == b["result"]["n_bunches"]
    assert a["result"]["drops"] == b["result"]["drops"]
    np.testing.assert_array_equal(a["offsets"], b["offsets"])
    np.testing.assert_array_equal(a["ids"], b["ids"])
    ra, rb = a["rec"].astype(np.float64), b["rec"].astype(np.float64)
    np.testing.assert_allclose(ra[:, :2], rb[:, :2], rtol=0, atol=5e-5)
    np.testing.assert_allclose(ra[:, 2:4], rb[:, 2:4], rtol=0, atol=1e-7)
    np.testing.assert_allclose(ra[:, 4], rb[:, 4], rtol=4 * F32, atol=1e-4)
    np.testing.assert_allclose(ra[:, 5:], rb[:, 5:], rtol=2 * F32, atol=0)


def test_curved_graph_replay_and_launch_shapes():
    """Deterministic output: other launch shapes and graph replays give the same
    bytes as an eager run."""
    import torch
    wl = synth.inclined(70.0, 6000)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED, earth_radius=R_EARTH)
    eager = gpu_run(wl, ckv.CKV_MIXED, earth_radius=R_EARTH, capacity=65536)
    for kw in (dict(waves_per_group=4), dict(waves_per_group=2, grid=97)):
        other = gpu_run(wl, ckv.CKV_MIXED, earth_radius=R_EARTH, capacity=65536, **kw)
        np.testing.assert_array_equal(other["offsets"], eager["offsets"])
        np.testing.assert_array_equal(other["rec"].view(np.uint32), eager["rec"].view(np.uint32))
    gr = ckv.GraphRunner(ckv.Runner(d, atmo, tels, p, 65536))
    for rep in range(3):
        gr.runner.records.fill_(float("nan"))
        torch.cuda.synchronize()
        out = gr.replay()
        torch.cuda.synchronize()
        n = out.result()["n_records"]
        np.testing.assert_array_equal(out.tel_offsets.cpu().numpy(), eager["offsets"])
        np.testing.assert_array_equal(out.records[:n].cpu().numpy().view(np.uint32),
                                      eager["rec"].view(np.uint32))


def test_curved_streamed_chunks_equal_one_shot():
    """The streamer plans ranges from ckv_count (curved midpoint altitudes) and
    resumes a range that overflows; per telescope the chunks concatenate to the
    one-shot curved output, bit for bit."""
    import torch
    wl = synth.inclined(70.0, 20000)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED, earth_radius=R_EARTH)
    one = gpu_run(wl, ckv.CKV_MIXED, handles_=(atmo, tels), earth_radius=R_EARTH)
    n_tel = tels.n
    st = ckv.Streamer(d, atmo, tels, p, chunk_records=300, first_ratio=0.001, plan_block=64)
    got = [[] for _ in range(n_tel)]
    n_chunks = 0
    for ch in st.chunks():
        n_chunks += 1
        off = ch.tel_offsets.cpu().numpy()
        rec = ch.records.cpu().numpy().copy()
        ids = ch.ids.cpu().numpy().copy()
        ids[:, 0] += ch.begin
        for t in range(n_tel):
            got[t].append((rec[off[t]:off[t + 1]], ids[off[t]:off[t + 1]]))
    torch.cuda.synchronize()
    say(f"[gpu] curved streamed: {n_chunks} chunks, {st.n_resumed} resumed, {st.n_reruns} rerun")
    assert n_chunks >= 5
    o = one["offsets"]
    for t in range(n_tel):
        rec = np.concatenate([x[0] for x in got[t]])
        ids = np.concatenate([x[1] for x in got[t]])
        np.testing.assert_array_equal(rec.view(np.uint32), one["rec"][o[t]:o[t + 1]].view(np.uint32))
        np.testing.assert_array_equal(ids, one["ids"][o[t]:o[t + 1]])


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_curved_several_showers_one_launch(precision):
    """Three inclined showers of different sizes, zeniths, azimuths and cores in one
    curved launch: per (shower, telescope) lists, counts and drops as the oracle."""
    atmo = synth.layered_atmosphere()
    parts = [synth.shower_segments(s, n, atmo, zenith_deg=z, azimuth_deg=az, core=c, xmax=400.0)
             for s, n, z, az, c in ((0, 5000, 60.0, 0.0, (0.0, 0.0)),
                                    (1, 12000, 72.0, 135.0, (300.0, -200.0)),
                                    (2, 3000, 80.0, 250.0, (-500.0, 400.0)))]
    segs = synth.Segments.concat(parts)
    wl = synth.Workload("curved_mix", atmo, synth.telescopes_disk(), segs)
    cfg = oracle.Config.from_workload(wl, earth_radius=R_EARTH)
    r = oracle.run(cfg, segs, nthreads=16)
    g = gpu_run(wl, precision, earth_radius=R_EARTH, capacity=4 * len(r.seg) + 4096)
    res = g["result"]
    assert res["error"] == 0 and res["overflow"] == 0, res
    assert res["n_bunches"] == r.n_bunches and res["drops"] == r.drops, (res, r.drops)
    if precision == ckv.CKV_FP64:
        np.testing.assert_array_equal(g["offsets"], r.offsets)
    rep = compare_records(wl, cfg, r, g, precision)
    say(f"[gpu] curved 3 showers prec={precision}: hits={res['n_hits']} {rep}")


def test_curved_full_size_sampled():
    """The 70-degree TeV shower at the benchmark's size (2e6 steps, 5.2e7 bunches),
    curved, mixed, in the benchmark's launch shape: every step's bunch count
    against the oracle, and the records of every 97th step (with their original
    random numbers) against the oracle's curved run of those steps."""
    import torch
    wl = synth.inclined(70.0)
    assert wl.segs.n == 2_000_000
    cfg = oracle.Config.from_workload(wl, earth_radius=R_EARTH)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED, earth_radius=R_EARTH, tile_segments=32)
    n_b = ckv.count(d, atmo, p).cpu().numpy()
    nb_o = oracle.segment_details(cfg, wl.segs)["n_b"].astype(np.int64)
    np.testing.assert_array_equal(n_b, nb_o)
    r = ckv.Runner(d, atmo, tels, p, 1 << 20)
    out = r.run()
    torch.cuda.synchronize()
    res = out.result()
    assert res["error"] == 0 and res["overflow"] == 0 and res["n_bunches"] == int(nb_o.sum())
    n = res["n_records"]
    off = out.tel_offsets.cpu().numpy()
    rec = out.records[:n].cpu().numpy()
    ids = out.ids[:n].cpu().numpy()
    idx = np.arange(0, wl.segs.n, 97)
    keep = np.isin(ids[:, 0], idx)
    counts = np.diff(off)
    group = np.repeat(np.arange(len(counts)), counts)[keep]
    off_k = np.zeros(len(counts) + 1, dtype=np.int64)
    off_k[1:] = np.cumsum(np.bincount(group, minlength=len(counts)))
    sub = wl.segs.take(idx)
    ores = oracle.run(cfg, sub, nthreads=16, seg_id=idx)
    rep = compare_records(wl, cfg, ores, dict(offsets=off_k, rec=rec[keep], ids=ids[keep]),
                          ckv.CKV_MIXED, segs=sub, seg_map=idx)
    say(f"[gpu] curved 70 deg full size: {res['n_bunches']} bunches, {n} records; sampled {rep}")
