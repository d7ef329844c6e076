"""Host-side bookkeeping of the binding and the input generators (no GPU)."""

import numpy as np

from paper_2006_14927_amd import ckv, synth


def _three_showers():
    atmo = synth.layered_atmosphere()
    parts = [synth.shower_segments(s, n, atmo, zenith_deg=20.0) for s, n in ((0, 50), (1, 7), (2, 40))]
    return synth.Segments.concat(parts)


def test_segment_view_keeps_shower_ids_and_step_indices():
    segs = _three_showers()
    d = ckv.DeviceSegments(segs, device="cpu", seg_id_base=[0, 3, 0])
    for a, b in ((0, 97), (10, 55), (50, 57), (52, 53), (56, 90), (57, 97), (0, 1)):
        v = d.view(a, b)
        s0, s1 = v.shower_range
        off = segs.seg_offsets
        assert off[s0] <= a < off[s0 + 1] and off[s1 - 1] < b <= off[s1]
        assert v.n == b - a and v.n_showers == s1 - s0
        so = v.seg_offsets.numpy()
        assert so[0] == 0 and so[-1] == b - a and np.all(np.diff(so) >= 0)
        # global step index of every step in the view -> (shower, index in shower + base)
        for j in range(v.n):
            loc = int(np.searchsorted(so, j, side="right") - 1)
            s = s0 + loc
            want = (a + j) - off[s] + [0, 3, 0][s]
            assert v.base_host[loc] + (j - so[loc]) == want
        np.testing.assert_array_equal(v.t["x0"].numpy(), segs.x0[a:b])
        np.testing.assert_array_equal(v.shower_ids.numpy(), segs.shower_ids[s0:s1].view(np.int32))


def test_take_shower_and_concat():
    segs = _three_showers()
    one = segs.take_shower(2, np.array([0, 5, 39]))
    assert one.n == 3 and one.t_ref[0] == segs.t_ref[2] and one.shower_ids[0] == 2
    np.testing.assert_array_equal(one.h0, segs.h0[[57, 62, 96]])
    parts = [segs.take_shower(s, np.arange(n)) for s, n in enumerate((50, 7, 40))]
    back = synth.Segments.concat(parts, consume=True)
    assert all(p is None for p in parts)
    for f in segs.FIELDS + ("ptype", "seg_offsets", "t_ref", "shower_ids"):
        np.testing.assert_array_equal(getattr(back, f), getattr(segs, f))


def test_threaded_generation_is_deterministic():
    a = synth.batched_showers(12, seg_scale=2e-3, workers=1)
    b = synth.batched_showers(12, seg_scale=2e-3, workers=4)
    for f in a.segs.FIELDS + ("ptype", "seg_offsets", "t_ref", "shower_ids"):
        np.testing.assert_array_equal(getattr(a.segs, f), getattr(b.segs, f))


def test_large_shower_blocks():
    atmo = synth.layered_atmosphere()
    old = synth.BLOCK_SEGMENTS
    try:
        synth.BLOCK_SEGMENTS = 1000
        big = synth.large_shower(3, 2500, atmo, workers=3, zenith_deg=40.0, muon_fraction=0.1)
    finally:
        synth.BLOCK_SEGMENTS = old
    assert big.n == 2500 and big.n_showers == 1 and big.shower_ids[0] == 3
    blk = synth.shower_segments(3, 1000, atmo, block=1, zenith_deg=40.0, muon_fraction=0.1)
    np.testing.assert_array_equal(big.x0[1000:2000], blk.x0)
    assert np.all(np.isfinite(big.h0))


def test_stream_range_planning():
    """Ranges respect the crossing budget at block granularity, always advance,
    and stay inside the input."""
    st = ckv.Streamer.__new__(ckv.Streamer)
    rng = np.random.default_rng(3)
    n = 100_003
    nb = rng.integers(0, 200, size=n)
    nb[5000:9000] = 0
    cum = np.concatenate([[0], np.cumsum(nb)])
    st.block = 4096
    st.plan_at = np.concatenate([[0], np.minimum(np.arange(4096, n + 4096, 4096), n)])
    st.plan_cum = cum[st.plan_at]
    st.capacity, st.max_range = 50_000, n

    class D:
        pass
    st.dsegs = D()
    st.dsegs.n = n
    for ratio in (1e-3, 0.05, 0.5, 20.0):
        st.ratio = ratio
        a = 0
        while a < n:
            b = st._range_end(a)
            assert a < b <= n
            if b - a > 1 and b % 4096 == 0:
                assert (cum[b] - cum[a]) * ratio <= 0.8 * st.capacity + 1e-9
            a = b


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before any device is touched."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
