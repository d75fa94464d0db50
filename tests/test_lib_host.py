"""Host-side tests of the library (no GPU): the C ABI loads and exports every
symbol its header declares; the library's graph path (Levy sampling, SLO
colouring) is bit-identical to the oracle's; the colour-sorted CSR is a
faithful relabelling of the edge list; argument errors are reported."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1211_3991_amd as xy
from paper_1211_3991_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "xy_levy.h")).read()
    declared = set(re.findall(r"^\s*(?:xy_status|void|const char \*)\s*(xy_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 17
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(_lib.raw(), name), name


@pytest.mark.parametrize("L,z,rho,seed", [(16, 6, 3.5, 1), (128, 6, 3.5, 0), (128, 6, 3.5, 63), (256, 6, 3.5, 7),
                                          (32, 6, 2.5, 2), (64, 6, 4.5, 33), (512, 6, 2.5, 0), (16, 4, 60.0, 3),
                                          (32, 6, 0.0, 5)])
def test_graph_bitwise_equal_to_oracle(L, z, rho, seed):
    g = xy.Graph.levy(L, z, rho, seed)
    ex = g.export()
    e, att = oracle.levy_graph(L, z, rho, seed)
    assert g.attempts == att
    assert np.array_equal(ex["edges"], e)
    col, q = oracle.slo_colour(L * L, e)
    assert g.n_colours == q
    assert np.array_equal(ex["colour"], col)


@pytest.mark.parametrize("L,z,rho,seed", [(16, 6, 3.5, 1), (17, 4, 2.5, 3), (32, 4, 14 / 3, 5), (20, 6, 0.0, 2)])
def test_free_boundary_graph_bitwise_equal_to_oracle(L, z, rho, seed):
    g = xy.Graph.levy(L, z, rho, seed, boundary="free")
    e, att = oracle.levy_graph(L, z, rho, seed, boundary="free")
    assert g.attempts == att and np.array_equal(g.export()["edges"], e)


def test_free_boundary_errors():
    for L in (1, 5000):
        with pytest.raises(xy.XYError):
            xy.Graph.levy(L, 4, 2.5, 1, boundary="free")
    with pytest.raises(xy.XYError):
        xy.Graph.levy(16, 4, 60.0, 1, boundary="free")      # too few short pairs: attempt cap


def test_colour_sorted_csr_is_a_relabelling():
    L = 64
    n = L * L
    g = xy.Graph.levy(L, 6, 3.5, 11)
    ex = g.export()
    perm, off, rp, col, colour = ex["perm"], ex["colour_off"], ex["row_ptr"], ex["col"], ex["colour"]
    assert sorted(perm) == list(range(n))
    # colour-major: class c occupies [off[c], off[c+1]) in lattice order
    for c in range(g.n_colours):
        cls = perm[off[c]:off[c + 1]]
        assert np.all(colour[cls] == c) and np.all(np.diff(cls) > 0)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    got = set()
    for k in range(n):
        row = col[rp[k]:rp[k + 1]]
        assert np.all(np.diff(row) > 0)                       # ascending, no repeats
        for j in row:
            got.add((min(perm[k], perm[j]), max(perm[k], perm[j])))
    want = {(min(a, b), max(a, b)) for a, b in ex["edges"]}
    assert got == want and rp[-1] == 2 * g.m
    # same-colour sites are never linked (the colouring is proper)
    cm = np.repeat(np.arange(g.n_colours), np.diff(off))
    src = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(cm[src] != cm[col])


def test_from_edges_and_errors():
    g = xy.Graph.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert (g.n, g.m, g.n_colours) == (4, 4, 2)
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.from_edges(3, [(0, 1), (1, 0)])
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.from_edges(3, [(0, 0)])
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.from_edges(3, [(0, 5)])
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.levy(15, 6, 3.5, 0)          # odd L
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.levy(16, 6, -1.0, 0)
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.levy(4, 15, 1.0, 0)          # z >= N - 1
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.levy(2, 3, 1.0, 0)           # z >= N - 1 with N = 4
    with pytest.raises(xy.XYError, match="EINVAL"):
        xy.Graph.from_edges(2, [(0, 1)], L=4, coords=[(0, 0), (4, 0)])   # coordinate outside [0, L)


def test_batch_argument_errors_without_device():
    """Argument checks of the batch entry points happen before any device call."""
    import ctypes
    g = xy.Graph.levy(8, 6, 3.5, 0)
    garr = (ctypes.c_void_p * 1)(g._h.value)
    sz = _lib.Sizes()
    raw = _lib.raw()
    assert raw.xy_batch_sizes(garr, 1, 0, 1, 0, ctypes.byref(sz)) == _lib.XY_EINVAL        # n_T = 0
    assert raw.xy_batch_sizes(garr, 1, 257, 1, 0, ctypes.byref(sz)) == _lib.XY_EINVAL      # n_T > 256
    assert raw.xy_batch_sizes(garr, 1, 4, 7, 0, ctypes.byref(sz)) == _lib.XY_EINVAL        # precision
    assert raw.xy_batch_sizes(garr, 0, 4, 1, 0, ctypes.byref(sz)) == _lib.XY_EINVAL        # no graphs
    assert raw.xy_batch_sizes(garr, 1, 4, 1, 5, ctypes.byref(sz)) == _lib.XY_OK
    assert sz.state_bytes >= 64 * 4 * 2 and sz.obs_bytes >= 5 * 4 * 8 * 8
    h = ctypes.c_void_p()
    T = np.array([1.0, -1.0, 2.0, 3.0])
    seeds = np.zeros(1, np.uint64)
    st = raw.xy_batch_init(ctypes.byref(h), garr, 1, 4, T.ctypes.data_as(ctypes.c_void_p), 1,
                           seeds.ctypes.data_as(ctypes.c_void_p), 0, None, None, None, None, None)
    assert st == _lib.XY_EINVAL and b"temperatures" in raw.xy_last_error()
    T = np.array([1.0, 1.5, 2.0, 3.0])
    st = raw.xy_batch_init(ctypes.byref(h), garr, 1, 4, T.ctypes.data_as(ctypes.c_void_p), 1,
                           seeds.ctypes.data_as(ctypes.c_void_p), 0, None, None, None, None, None)
    assert st == _lib.XY_EINVAL and b"NULL device buffer" in raw.xy_last_error()
    assert raw.xy_sweep(None, None, 1, 5, 1, 1, None) == _lib.XY_EINVAL
    assert raw.xy_measure(None, None, None) == _lib.XY_EINVAL


def test_single_hip_runtime_in_process():
    """The library shares PyTorch's HIP runtime (one libamdhip64 mapped)."""
    maps = open("/proc/self/maps").read()
    paths = {ln.split()[-1] for ln in maps.splitlines() if "libamdhip64" in ln}
    assert len(paths) == 1, paths


def test_noalloc_walk_rejects_oversized_input_on_the_host():
    """xy_random_walk_noalloc checks its arguments and the static workspace's
    limit (32 MiB of walk records) before any device call."""
    import ctypes
    n = 2048 * 2048                                   # 16 B of record per site: 64 MiB
    g = xy.Graph.from_edges(n, np.zeros((0, 2), np.int32), L=2048)
    garr = (ctypes.c_void_p * 1)(g._h.value)
    seeds = np.zeros(1, np.uint64)
    raw = _lib.raw()
    hist = ctypes.c_void_p(256)                       # never dereferenced: the call returns first
    assert raw.xy_random_walk_noalloc(garr, 1, 1, 1, ctypes.c_void_p(seeds.ctypes.data), 1, hist, None,
                                      None) == _lib.XY_EINVAL
    assert b"static workspace" in raw.xy_last_error()
    assert raw.xy_random_walk_noalloc(garr, 1, -1, 1, ctypes.c_void_p(seeds.ctypes.data), 1, hist, None,
                                      None) == _lib.XY_EINVAL
    assert raw.xy_random_walk_noalloc(garr, 1, 1, 1, None, 1, hist, None, None) == _lib.XY_EINVAL
