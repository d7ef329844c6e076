"""ckv_run_noalloc (the workspace-free variant of ckv_run, for callers that
cannot allocate device memory) against ckv_run through the C ABI: identical
records, ids, offsets and reports on two calls in a row, the second on a
smaller input, so a stale workspace from the first call would show."""

import ctypes as C

import numpy as np
import pytest

from paper_2006_14927_amd import ckv, synth

from gpu_helpers import handles, params, say

pytestmark = pytest.mark.gpu


def _outputs(n_showers, n_tel, capacity):
    import torch
    return ckv._OutBuf(capacity, n_showers * n_tel, True, "cuda")


def _host(out, n_groups):
    import torch
    torch.cuda.synchronize()
    res = out.result()
    n = int(res["n_records"])
    return (res, out.records[:n].cpu().numpy().copy(), out.ids[:n].cpu().numpy().copy(),
            out.tel_offsets[:n_groups + 1].cpu().numpy().copy())


def _both(wl, segs, precision, capacity):
    import torch
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(segs)
    p = params(wl, precision)
    L = ckv.lib()
    ng = d.n_showers * tels.n
    need = L.ckv_noalloc_workspace_size(d.n, d.n_showers, tels.n, capacity, C.byref(p))
    assert 0 < need <= ckv.NOALLOC_SCRATCH_BYTES
    ref = ckv.Runner(d, atmo, tels, p, capacity, want_ids=True)
    r_ref = ref.run()
    a = _host(r_ref, ng)
    out = _outputs(d.n_showers, tels.n, capacity)
    segs_c, show_c, o = d.c_segments(), d.c_showers(), out.c_output(capacity)
    stream = torch.cuda.current_stream()
    say(f"[gpu] ckv_run_noalloc {wl.name} n={d.n} prec={precision} cap={capacity} ws={need}")
    rc = L.ckv_run_noalloc(C.byref(segs_c), C.byref(show_c), C.byref(p), atmo.handle, tels.handle,
                           C.byref(o), None, C.c_void_p(stream.cuda_stream))
    assert rc == 0, L.ckv_last_error()
    b = _host(out, ng)
    return a, b


def _same(a, b):
    ra, reca, ida, offa = a
    rb, recb, idb, offb = b
    assert ra == rb
    assert ra["error"] == 0 and ra["overflow"] == 0 and ra["n_records"] > 0
    np.testing.assert_array_equal(offa, offb)
    np.testing.assert_array_equal(ida, idb)
    assert reca.tobytes() == recb.tobytes()


@pytest.mark.parametrize("precision", [ckv.CKV_FP64, ckv.CKV_MIXED])
def test_noalloc_matches_run_twice_second_smaller(precision):
    wl = synth.batched_showers(6, seg_scale=0.02)
    first = _both(wl, wl.segs, precision, capacity=wl.segs.n * 4)
    _same(*first)
    small = wl.segs.take(np.arange(0, wl.segs.n // 3))
    second = _both(wl, small, precision, capacity=max(1024, small.n * 2))
    _same(*second)
    assert second[0][0]["n_bunches"] < first[0][0]["n_bunches"]


def test_noalloc_refuses_a_run_larger_than_its_array():
    """Checked on the host before anything is enqueued: no GPU work starts."""
    wl = synth.vertical_gamma(100)
    atmo, tels = handles(wl)
    d = ckv.DeviceSegments(wl.segs)
    p = params(wl, ckv.CKV_MIXED)
    L = ckv.lib()
    cap = ckv.NOALLOC_SCRATCH_BYTES // 16          # records alone exceed the array
    assert L.ckv_noalloc_workspace_size(d.n, d.n_showers, tels.n, cap, C.byref(p)) > \
        ckv.NOALLOC_SCRATCH_BYTES
    out = ckv._Output(None, None, cap, None, None)
    segs_c, show_c = d.c_segments(), d.c_showers()
    rc = L.ckv_run_noalloc(C.byref(segs_c), C.byref(show_c), C.byref(p), atmo.handle, tels.handle,
                           C.byref(out), None, None)
    assert rc == -3 and b"static scratch" in L.ckv_last_error()
