"""The allocation-free walk entry point (xy_random_walk_noalloc), through the
C ABI: its histograms equal xy_random_walk's entry by entry (integer work on
counter-based draws), on two calls in a row, the second with smaller graphs
(the static workspace keeps the first call's records beyond what the second
stages), for both start rules; a set of graphs larger than the workspace is
rejected with a clear error and leaves the next call correct."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1211_3991_amd as xy  # noqa: E402
from paper_1211_3991_amd import _lib  # noqa: E402


def _noalloc_raw(graphs, n_walkers, n_steps, seeds, start_mode):
    """xy_random_walk_noalloc called through ctypes directly."""
    G = len(graphs)
    garr = (ctypes.c_void_p * G)(*[g._h.value for g in graphs])
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    hist = torch.full((G, n_steps + 1), -1, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    rc = _lib.raw().xy_random_walk_noalloc(garr, G, n_walkers, n_steps, ctypes.c_void_p(seeds.ctypes.data),
                                           start_mode, ctypes.c_void_p(hist.data_ptr()),
                                           ctypes.c_void_p(st.cuda_stream), None)
    torch.cuda.synchronize()
    return rc, hist


@pytest.mark.parametrize("start_mode,start", [(1, "degree3"), (0, "centre")])
def test_noalloc_walk_equals_walk_on_two_calls(start_mode, start):
    calls = [([xy.Graph.levy(96, 4, 3.5, s) for s in range(6)], 3000, 700, np.arange(6) + 11),
             ([xy.Graph.levy(32, 6, 2.5, 9)], 257, 300, np.array([5]))]
    for graphs, W, T, seeds in calls:
        ref = xy.random_walk(graphs, W, T, seeds=seeds, start=start)
        torch.cuda.synchronize()
        rc, got = _noalloc_raw(graphs, W, T, seeds, start_mode)
        assert rc == _lib.XY_OK, _lib.raw().xy_last_error()
        assert torch.equal(got, ref), (len(graphs), W, T)
        assert int(got[0, 0]) == W
        # the binding's wrapper gives the same
        assert torch.equal(xy.random_walk_noalloc(graphs, W, T, seeds=seeds, start=start), ref)


def test_noalloc_walk_rejects_graphs_beyond_the_workspace():
    big = [xy.Graph.levy(1024, 4, 3.5, 1), xy.Graph.levy(1024, 4, 3.5, 2)]   # about 40 MB of walk records
    nbytes = ctypes.c_size_t()
    garr = (ctypes.c_void_p * 2)(*[g._h.value for g in big])
    _lib.call("xy_walk_bytes", garr, 2, ctypes.byref(nbytes))
    assert nbytes.value > 32 << 20
    rc, hist = _noalloc_raw(big, 10, 5, [1, 2], 1)
    assert rc == _lib.XY_EINVAL and b"static workspace" in _lib.raw().xy_last_error()
    assert int(hist.min()) == -1 and int(hist.max()) == -1        # nothing written
    small = [xy.Graph.levy(32, 6, 3.5, 4)]
    ref = xy.random_walk(small, 100, 50, seeds=[3])
    assert torch.equal(xy.random_walk_noalloc(small, 100, 50, seeds=[3]), ref)
