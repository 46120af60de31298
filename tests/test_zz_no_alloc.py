"""cbaa_merge_restore_noalloc, the window end for callers that cannot
allocate device memory, against cbaa_merge_restore with a caller buffer.

Two calls in a row share the library's per-device scratch array: a two-router
window with the merged cube not stored, then a smaller single-cube window
with a smaller capacity and the merge stored. Each call's list and counters
must equal those of cbaa_merge_restore on the same cubes (and the oracle's
hosts), so nothing left in the array by the first call leaks into the second."""

import numpy as np
import pytest

import oracle as O
import tracegen
from conftest import default_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06207_amd import cbaa
    cbaa.lib()
    return cbaa


def _say(*a):
    print("[case]", *a, flush=True)


def _with_buffer(cb, p, dst, srcs, cap):
    import torch
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * cb.HOST_BYTES, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    cb.cbaa_merge_restore(p, dst, srcs, 1024.0, cb.THR_THM2, rs, out, cap, st)
    torch.cuda.synchronize()
    return cb.host_list(out, min(int(st[0]), cap)), st.cpu().numpy().copy()


def _no_alloc(cb, p, dst, srcs, cap):
    import torch
    out = torch.full((cap * cb.HOST_BYTES,), 0xAB, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    cb.cbaa_merge_restore_noalloc(p, dst, srcs, 1024.0, cb.THR_THM2, out, cap, st)
    torch.cuda.synchronize()
    return cb.host_list(out, min(int(st[0]), cap)), st.cpu().numpy().copy()


def _same(a, b):
    assert a.size == b.size
    for f in ("ip", "zeros", "cs", "flags"):
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["est"], b["est"])     # same kernels, same inputs: identical doubles


def test_noalloc_matches_caller_scratch_twice(cb):
    import torch
    p = default_params()
    # call 1: a 1M-packet window split over two routers, merge not stored
    _say("noalloc call 1: 2 routers, 1M packets, dst=None, capacity 4096")
    t1 = tracegen.window_small(5)
    cubes = []
    for q in tracegen.split_routers(t1.pairs, 2, seed=3):
        c = cb.new_cube(p)
        cb.cbaa_update(p, c, cb.pairs_to_device(q), cb.SIDE_SRC)
        cubes.append(c)
    want1, st_want1 = _with_buffer(cb, p, None, cubes, 4096)
    got1, st_got1 = _no_alloc(cb, p, None, cubes, 4096)
    _same(got1, want1)
    assert np.array_equal(st_got1, st_want1)
    ref1, _ = O.restore(p, O.cube_of(p, t1.pairs, 0), 1024.0)
    assert np.array_equal(got1["ip"], ref1["ip"])
    assert got1.size > 10

    # call 2: a smaller window in one cube, stored merge, smaller capacity
    _say("noalloc call 2: 1 cube, 250k packets, stored merge, capacity 512")
    t2 = tracegen.make_window(250_000, 30_000, 6, 1_500, 6_000, dup_frac=0.05, seed=77)
    c2 = cb.new_cube(p)
    cb.cbaa_update(p, c2, cb.pairs_to_device(t2.pairs), cb.SIDE_SRC)
    d_want = cb.new_cube(p, init=False)
    d_got = cb.new_cube(p, init=False)
    want2, st_want2 = _with_buffer(cb, p, d_want, [c2], 512)
    got2, st_got2 = _no_alloc(cb, p, d_got, [c2], 512)
    _same(got2, want2)
    assert np.array_equal(st_got2, st_want2)
    assert torch.equal(d_got, d_want)
    ref2, _ = O.restore(p, O.cube_of(p, t2.pairs, 0), 1024.0)
    assert np.array_equal(got2["ip"], ref2["ip"])
    assert 0 < got2.size < got1.size


def test_noalloc_rejects_capacity_beyond_its_array(cb):
    import ctypes as C
    import torch
    p = default_params()
    cap = 4_000_000
    assert cb.cbaa_restore_scratch_bytes(p, cap) > cb.NOALLOC_SCRATCH_BYTES
    c = cb.new_cube(p)
    out = torch.empty(cap * cb.HOST_BYTES, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    arr = (C.c_void_p * 1)(c.data_ptr())
    rc = cb.lib().cbaa_merge_restore_noalloc(C.byref(cb._cfg(p)), None, arr, 1, 1024.0, 0, 0,
                                             out.data_ptr(), cap, st.data_ptr(), None)
    assert rc == cb.CBAA_ESCRATCH
    assert "no-allocation" in cb.cbaa_last_error()
