"""MI355X-native Monte Carlo of the XY model on dilute Levy graphs.

Ibanez Berganza & Leuzzi, "Critical behavior of the XY model in complex
topologies" (arXiv:1211.3991): equilibrium Metropolis + over-relaxation
sweeps with parallel tempering (App. B) of O(2) spins on Levy graphs
(Sec. 2, Eq. Levyi), measuring E, |m|^2, |m|^4 and chi(k_min) (Sec. 3).

This package is a thin Python face of ``libxylevy.so`` (C ABI declared in
``include/xy_levy.h``): ``Graph`` wraps the host graph path (sampling,
smallest-last colouring, colour-sorted CSR), ``Batch`` wraps the device
path (HIP kernels for gfx950) and ``random_walk`` the self-return histograms
of random walkers (App. A).  PyTorch only provides device memory and the
stream; every step of the computation runs in the library.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import XY_FIX16, XY_FP64, XY_NOBS, XYError

__all__ = ["Graph", "Batch", "random_walk", "random_walk_noalloc", "XYError", "XY_FP64", "XY_FIX16", "XY_NOBS", "OBS_NAMES"]

OBS_NAMES = ("E", "m2", "m4", "Fx", "Fy", "mx", "my", "pad")
_PREC = {"fp64": XY_FP64, "fix16": XY_FIX16}


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class Graph:
    """A host graph handle (xy_graph)."""

    def __init__(self, handle):
        self._free = _lib.raw().xy_graph_free
        self._h = ctypes.c_void_p(handle)
        n, m, q, md = (ctypes.c_int() for _ in range(4))
        att = ctypes.c_int64()
        _lib.call("xy_graph_info", self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(q),
                  ctypes.byref(md), ctypes.byref(att))
        self.n, self.m, self.n_colours, self.max_degree, self.attempts = n.value, m.value, q.value, md.value, att.value

    @classmethod
    def levy(cls, L, z, rho, seed, boundary="periodic"):
        """Dilute Levy graph on the L x L lattice, periodic or free boundaries."""
        fn = {"periodic": "xy_graph_levy", "free": "xy_graph_levy_free"}[boundary]
        h = ctypes.c_void_p()
        _lib.call(fn, int(L), int(z), float(rho), int(seed), ctypes.byref(h))
        g = cls(h.value)
        g.L = int(L)
        return g

    @classmethod
    def from_edges(cls, n, edges, L=None, coords=None):
        e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        c = None if coords is None else np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 2)
        L = int(L if L is not None else n)
        h = ctypes.c_void_p()
        _lib.call("xy_graph_from_edges", int(n), e.shape[0], _ptr(e) if e.size else None, _ptr(c), L,
                  ctypes.byref(h))
        g = cls(h.value)
        g.L = L
        return g

    def export(self):
        e = np.empty((self.m, 2), np.int32)
        colour = np.empty(self.n, np.int32)
        perm = np.empty(self.n, np.int32)
        off = np.empty(self.n_colours + 1, np.int32)
        rp = np.empty(self.n + 1, np.int32)
        col = np.empty(2 * self.m, np.int32)
        _lib.call("xy_graph_export", self._h, _ptr(e), _ptr(colour), _ptr(perm), _ptr(off), _ptr(rp), _ptr(col))
        return {"edges": e, "colour": colour, "perm": perm, "colour_off": off, "row_ptr": rp, "col": col}

    def __del__(self):
        # the free function is bound at creation: module globals may already
        # be gone when the interpreter shuts down
        h, free = getattr(self, "_h", None), getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None


class Batch:
    """n_graphs samples x n_T temperatures on one GPU (xy_batch).

    Device buffers are torch uint8 tensors owned by this object; the library
    only receives their addresses.  All calls are enqueued on `stream`
    (default: torch's current stream on the device)."""

    def __init__(self, graphs, T, precision="fix16", seeds=None, max_records=0, device="cuda", stream=None):
        import torch
        self._torch = torch
        self.graphs = list(graphs)
        G = len(self.graphs)
        T = np.asarray(T, dtype=np.float64)
        if T.ndim == 1:
            T = np.tile(T, (G, 1))
        self.T = np.ascontiguousarray(T)
        self.G, self.R = G, self.T.shape[1]
        self.precision = precision
        self.max_records = int(max_records)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Batch needs a GPU device")
        seeds = np.arange(G, dtype=np.uint64) if seeds is None else np.asarray(seeds, dtype=np.uint64)
        self.seeds = np.ascontiguousarray(seeds)
        garr = (ctypes.c_void_p * G)(*[g._h.value for g in self.graphs])
        sz = _lib.Sizes()
        _lib.call("xy_batch_sizes", garr, G, self.R, _PREC[precision], self.max_records, ctypes.byref(sz))
        self.sizes = sz

        def buf(nbytes):
            t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            if t.data_ptr() % 256:
                raise RuntimeError("device buffer is not 256-byte aligned")
            return t
        self.d_state, self.d_graph = buf(sz.state_bytes), buf(sz.graph_bytes)
        self.d_work, self.d_obs = buf(sz.work_bytes), buf(sz.obs_bytes)
        self._stream = stream
        h = ctypes.c_void_p()
        _lib.call("xy_batch_init", ctypes.byref(h), garr, G, self.R, _ptr(self.T), _PREC[precision],
                  _ptr(self.seeds), self.max_records, ctypes.c_void_p(self.d_state.data_ptr()),
                  ctypes.c_void_p(self.d_graph.data_ptr()), ctypes.c_void_p(self.d_work.data_ptr()),
                  ctypes.c_void_p(self.d_obs.data_ptr()), self._s())
        self._h = h
        self._free = _lib.raw().xy_batch_free
        self._log = None

    def _s(self):
        st = self._stream if self._stream is not None else self._torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(st.cuda_stream)

    def sweep(self, n_sweeps, n_or=5, pt_every=1, meas_every=32, T=None):
        """n_sweeps sweeps; T (per-sample ladders [G, n_T] or one ladder [n_T])
        replaces the temperature of every index from this call on."""
        t = None
        if T is not None:
            t = np.asarray(T, dtype=np.float64)
            if t.ndim == 1:
                t = np.tile(t, (self.G, 1))
            if t.shape != (self.G, self.R):
                raise ValueError("T must be [n_T] or [n_graphs, n_T]")
            t = np.ascontiguousarray(t)
        _lib.call("xy_sweep", self._h, _ptr(t), int(n_sweeps), int(n_or), int(pt_every), int(meas_every),
                  self._s())
        if t is not None:
            self.T = t

    def use_graph(self, chunk):
        _lib.call("xy_batch_use_graph", self._h, int(chunk))

    def set_fix16_form(self, trig=2, allow_unit=True, force_global=False):
        """(cos, sin) form and spin storage of the fixed-point sweep (see xy_levy.h)."""
        _lib.call("xy_batch_set_fix16_form", self._h, int(trig), int(bool(allow_unit)), int(bool(force_global)),
                  self._s())

    def set_phase_streams(self, n, slices=1):
        """Stream groups of the phase-form samples: n streams (1..4) times
        `slices` groups per stream, the slices swept one after the other
        (n * slices <= 8); the trajectory does not depend on it."""
        _lib.call("xy_batch_set_phase_groups", self._h, int(n), int(slices), self._s())

    def phase_streams(self):
        n = ctypes.c_int()
        _lib.call("xy_batch_phase_streams", self._h, ctypes.byref(n))
        return n.value

    def phase_slices(self):
        n, sl = ctypes.c_int(), ctypes.c_int()
        _lib.call("xy_batch_phase_groups", self._h, ctypes.byref(n), ctypes.byref(sl))
        return sl.value

    def forms(self):
        """Storage form per sample: 1 site-major phase form, 0 workgroup per replica."""
        out = np.zeros(self.G, np.int32)
        _lib.call("xy_batch_forms", self._h, ctypes.c_void_p(out.ctypes.data))
        return out

    def autotune(self, sweeps=3, n_or=5, use_cache=True, pt_every=1, replay=True):
        """Times the fixed-point configurations on this batch and keeps the fastest."""
        from .autotune import autotune
        return autotune(self, sweeps=sweeps, n_or=n_or, use_cache=use_cache, pt_every=pt_every, replay=replay)

    def kernel_timing(self, enable=True):
        _lib.call("xy_kernel_timing", self._h, int(bool(enable)))

    def kernel_time(self):
        """(summed milliseconds, number of timed sweeps) of the dominant kernel."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _lib.call("xy_kernel_time", self._h, ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    def synchronize(self):
        st = self._stream if self._stream is not None else self._torch.cuda.current_stream(self.device)
        st.synchronize()

    def measure(self):
        """Observables of the current state: device tensor [G, n_T, 8] (float64),
        complete when this returns."""
        out = self._torch.empty((self.G, self.R, XY_NOBS), dtype=self._torch.float64, device=self.device)
        _lib.call("xy_measure", self._h, ctypes.c_void_p(out.data_ptr()), self._s())
        self.synchronize()
        return out

    def pt_energies(self):
        """Replica energies the last tempering step used, by slot: device
        tensor [G, n_T] (float64), complete when this returns."""
        out = self._torch.empty((self.G, self.R), dtype=self._torch.float64, device=self.device)
        _lib.call("xy_pt_energies", self._h, ctypes.c_void_p(out.data_ptr()), self._s())
        self.synchronize()
        return out

    def pt_swap(self):
        _lib.call("xy_pt_swap", self._h, self._s())

    def records(self):
        """Stored measurement records: device tensor [n_records, G, n_T, 8]."""
        n, _, _ = self.counters()
        rec = self.d_obs[: n * self.G * self.R * XY_NOBS * 8].view(self._torch.float64)
        return rec.view(n, self.G, self.R, XY_NOBS)

    def counters(self):
        nrec = ctypes.c_int()
        acc = np.zeros((self.G, self.R), np.uint64)
        tries = np.zeros((self.G, self.R), np.uint64)
        _lib.call("xy_get_counters", self._h, ctypes.byref(nrec), _ptr(acc), _ptr(tries), self._s())
        return nrec.value, acc, tries

    def get_state(self):
        """Host copy: fp64 -> list of [n_T, n, 2] float64; fix16 -> list of [n_T, n] uint16
        (lattice order), plus slot_of_T [G, n_T] and the sweep counter."""
        ns = [g.n for g in self.graphs]
        tot = sum(ns) * self.R
        if self.precision == "fp64":
            flat = np.empty(2 * tot, np.float64)
        else:
            flat = np.empty(tot, np.uint16)
        sot = np.empty((self.G, self.R), np.int32)
        sw = ctypes.c_uint32()
        _lib.call("xy_get_state", self._h, _ptr(flat), _ptr(sot), ctypes.byref(sw), self._s())
        out, off = [], 0
        for n in ns:
            k = n * self.R * (2 if self.precision == "fp64" else 1)
            a = flat[off:off + k]
            out.append(a.reshape(self.R, n, 2) if self.precision == "fp64" else a.reshape(self.R, n))
            off += k
        return out, sot, sw.value

    def set_state(self, states, slot_of_T=None, sweep=0):
        flat = np.concatenate([np.asarray(s).ravel() for s in states])
        flat = np.ascontiguousarray(flat, dtype=np.float64 if self.precision == "fp64" else np.uint16)
        sot = None if slot_of_T is None else np.ascontiguousarray(slot_of_T, dtype=np.int32)
        _lib.call("xy_set_state", self._h, _ptr(flat), _ptr(sot), int(sweep), self._s())

    def decision_log(self, max_sweeps):
        """Enables the Metropolis decision log for the next max_sweeps sweeps;
        returns the device tensor [max_sweeps, G, n_T, max_n] it fills."""
        max_n = max(g.n for g in self.graphs)
        self._log = self._torch.zeros((max_sweeps, self.G, self.R, max_n), dtype=self._torch.uint8,
                                      device=self.device)
        _lib.call("xy_decision_log", self._h, ctypes.c_void_p(self._log.data_ptr()), int(max_sweeps))
        return self._log

    def close(self):
        h, free = getattr(self, "_h", None), getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None

    def __del__(self):
        self.close()


_WALK_START = {"centre": 0, "degree3": 1}


def random_walk(graphs, n_walkers, n_steps, seeds=None, start="degree3", stream=None, timing=False):
    """Self-return histograms of random walkers on each graph (Sec. 2, spectral
    dimension; App. A): a torch.int64 [n_graphs, n_steps + 1] device tensor,
    entry (g, t) = walkers of graph g back at their start after t steps.
    start: "centre" (the lattice centre) or "degree3" (a random site of degree
    > 2 per walker).  The result is ready once `stream` (default: the current
    stream) has reached it.  timing=True waits for the walks and returns
    (histograms, milliseconds of the walk kernel)."""
    import torch
    G = len(graphs)
    seeds = np.arange(G, dtype=np.uint64) if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint64)
    if seeds.shape != (G,):
        raise ValueError("one seed per graph")
    garr = (ctypes.c_void_p * G)(*[g._h.value for g in graphs])
    nbytes = ctypes.c_size_t()
    _lib.call("xy_walk_bytes", garr, G, ctypes.byref(nbytes))
    st = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(st):
        d_graph = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device="cuda")
        hist = torch.empty((G, n_steps + 1), dtype=torch.int64, device="cuda")
    ms = ctypes.c_float()
    _lib.call("xy_random_walk", garr, G, int(n_walkers), int(n_steps), ctypes.c_void_p(seeds.ctypes.data),
              _WALK_START[start], ctypes.c_void_p(d_graph.data_ptr()), nbytes.value,
              ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(st.cuda_stream),
              ctypes.byref(ms) if timing else None)
    # d_graph is released to the caching allocator on `st`, after the walk in stream order
    return (hist, ms.value) if timing else hist


def random_walk_noalloc(graphs, n_walkers, n_steps, seeds=None, start="degree3", stream=None, timing=False):
    """random_walk through xy_random_walk_noalloc: the walk graphs are staged
    in the library's static device workspace (32 MiB per device) instead of a
    buffer allocated here; only the output histogram is allocated.  Calls
    that overlap on one device race on that workspace."""
    import torch
    G = len(graphs)
    seeds = np.arange(G, dtype=np.uint64) if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint64)
    if seeds.shape != (G,):
        raise ValueError("one seed per graph")
    garr = (ctypes.c_void_p * G)(*[g._h.value for g in graphs])
    st = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(st):
        hist = torch.empty((G, n_steps + 1), dtype=torch.int64, device="cuda")
    ms = ctypes.c_float()
    _lib.call("xy_random_walk_noalloc", garr, G, int(n_walkers), int(n_steps), ctypes.c_void_p(seeds.ctypes.data),
              _WALK_START[start], ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(st.cuda_stream),
              ctypes.byref(ms) if timing else None)
    return (hist, ms.value) if timing else hist
