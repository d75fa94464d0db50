"""Sequential FP64 CPU oracle for the XY model on dilute Levy graphs.

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the library.

This module is a ctypes wrapper around ``xy_oracle.c`` (plain C, FP64,
built with ``-ffp-contract=off``).  Each C function cites the passage of the
paper it follows (Ibanez Berganza & Leuzzi, arXiv:1211.3991):

* ``philox``            -- Philox4x32-10 (Salmon et al., SC'11), the counter-based
                           generator that replaces the paper's per-thread
                           lagged-Fibonacci generator (App. B, "Memory management").
* ``levy_graph``        -- dilute Levy graph, Sec. 2 Eq. (Levyi).
* ``slo_colour``        -- smallest-last-ordering colouring, App. B "Graph coloring".
* ``Sim``               -- Metropolis + over-relaxation + parallel tempering,
                           App. B "Improved equilibrium dynamics"; observables of
                           Sec. 3 (E, m, |m|^2, |m|^4, chi(k_min)).

Pins (the tests that tie each function to something other than itself) live
in ``tests/test_oracle_*.py``; parity status is stated in each test module.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OXY_LIB lets a mutation check point the tests at a deliberately broken copy.
_LIB_PATH = os.environ.get("OXY_LIB") or os.path.join(_HERE, "liboxy.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")

NOBS = 8
OBS_NAMES = ("E", "m2", "m4", "Fx", "Fy", "mx", "my", "pad")


def lib():
    """Loads liboxy.so, building it with gcc first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    L = ctypes.CDLL(_LIB_PATH)
    L.oxy_philox_batch.argtypes = [ctypes.c_int64, _u32p, _u32p, _u32p]
    L.oxy_philox_batch.restype = None
    L.oxy_levy_graph.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                 _i32p, ctypes.POINTER(ctypes.c_int64)]
    L.oxy_levy_graph.restype = ctypes.c_int
    L.oxy_levy_graph_free.argtypes = L.oxy_levy_graph.argtypes
    L.oxy_levy_graph_free.restype = ctypes.c_int
    L.oxy_levy_raw_draws.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                     ctypes.c_int64, _i32p]
    L.oxy_levy_raw_draws.restype = ctypes.c_int
    L.oxy_levy_weight_total.argtypes = [ctypes.c_int, ctypes.c_double]
    L.oxy_levy_weight_total.restype = ctypes.c_double
    L.oxy_slo_colour.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p]
    L.oxy_slo_colour.restype = ctypes.c_int
    L.oxy_random_walk.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.oxy_random_walk.restype = ctypes.c_int
    L.oxy_frozen_field_chain.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _f64p]
    L.oxy_frozen_field_chain.restype = ctypes.c_int
    L.oxy_or_move.argtypes = [ctypes.c_double, ctypes.c_double,
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.oxy_or_move.restype = None
    L.oxy_sim_create.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_uint64]
    L.oxy_sim_create.restype = ctypes.c_void_p
    L.oxy_sim_free.argtypes = [ctypes.c_void_p]
    L.oxy_sim_free.restype = None
    L.oxy_sim_n_colours.argtypes = [ctypes.c_void_p]
    L.oxy_sim_n_colours.restype = ctypes.c_int
    L.oxy_sim_init_random.argtypes = [ctypes.c_void_p]
    L.oxy_sim_init_random.restype = None
    L.oxy_sim_set_state.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_void_p, ctypes.c_uint32]
    L.oxy_sim_set_state.restype = None
    L.oxy_sim_get_state.argtypes = [ctypes.c_void_p, _f64p, _i32p, ctypes.POINTER(ctypes.c_uint32)]
    L.oxy_sim_get_state.restype = None
    L.oxy_sim_energy.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.oxy_sim_energy.restype = ctypes.c_double
    L.oxy_sim_measure.argtypes = [ctypes.c_void_p, _f64p]
    L.oxy_sim_measure.restype = None
    L.oxy_sim_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p]
    L.oxy_sim_run.restype = ctypes.c_int
    L.oxy_sim_pt_counts.argtypes = [ctypes.c_void_p, _i64p, _i64p]
    L.oxy_sim_pt_counts.restype = None
    _lib = L
    return L


def philox(ctr, key):
    """Philox4x32-10 of counters ctr[n,4] under keys key[n,2] -> uint32[n,4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    assert ctr.shape[0] == key.shape[0]
    out = np.empty_like(ctr)
    lib().oxy_philox_batch(ctr.shape[0], ctr, key, out)
    return out


def levy_graph(L, z, rho, seed, boundary="periodic"):
    """Edge list int32[M,2] in acceptance order, and the number of raw draws.
    boundary: "periodic" (the torus) or "free" (the open square)."""
    n = L * L
    m = n * z // 2
    edges = np.empty((m, 2), dtype=np.int32)
    att = ctypes.c_int64(0)
    fn = {"periodic": lib().oxy_levy_graph, "free": lib().oxy_levy_graph_free}[boundary]
    rc = fn(L, z, float(rho), seed, edges, ctypes.byref(att))
    if rc != 0:
        raise ValueError(f"oxy_levy_graph failed with {rc} (L={L}, z={z}, rho={rho})")
    return edges, att.value


def levy_raw_draws(L, rho, seed, n):
    """The first n raw draws (i, j) of the graph sampler, before rejection."""
    ij = np.empty((n, 2), dtype=np.int32)
    rc = lib().oxy_levy_raw_draws(L, float(rho), seed, n, ij)
    if rc != 0:
        raise MemoryError("oxy_levy_raw_draws")
    return ij


def levy_weight_total(L, rho):
    return lib().oxy_levy_weight_total(L, float(rho))


def slo_colour(n, edges):
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    colour = np.empty(n, dtype=np.int32)
    q = lib().oxy_slo_colour(n, edges.shape[0], edges, colour)
    if q < 0:
        raise MemoryError("oxy_slo_colour")
    return colour, q


def random_walk(n, edges, L, n_walkers, n_steps, seed, start_mode=1, return_starts=False):
    """Self-return histogram of random walkers (App. A): uint64[n_steps + 1],
    entry t = walkers at their start after t steps.  start_mode 0: the lattice
    centre; 1: a random site of degree > 2 per walker."""
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    hist = np.zeros(n_steps + 1, dtype=np.uint64)
    starts = np.zeros(max(n_walkers, 1), dtype=np.int32)
    rc = lib().oxy_random_walk(n, edges.shape[0], edges, L, n_walkers, n_steps, seed, start_mode,
                               hist.ctypes.data, starts.ctypes.data)
    if rc != 0:
        raise ValueError(f"oxy_random_walk: {rc}")
    return (hist, starts[:n_walkers]) if return_starts else hist


def frozen_field_chain(hx, hy, beta, seed, n_moves, or_every=0):
    ang = np.empty(n_moves, dtype=np.float64)
    acc = lib().oxy_frozen_field_chain(hx, hy, beta, seed, n_moves, or_every, ang)
    return ang, acc


def or_move(hx, hy, x, y):
    cx, cy = ctypes.c_double(x), ctypes.c_double(y)
    lib().oxy_or_move(hx, hy, ctypes.byref(cx), ctypes.byref(cy))
    return cx.value, cy.value


class Sim:
    """One graph simulated at n_T temperatures (one replica slot per T)."""

    def __init__(self, n, edges, colour, L, T, seed, coords=None):
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        colour = np.ascontiguousarray(colour, dtype=np.int32)
        self.T = np.ascontiguousarray(T, dtype=np.float64)
        self.n, self.m, self.nT = n, edges.shape[0], self.T.shape[0]
        self._coords = None
        cptr = None
        if coords is not None:
            self._coords = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 2)
            cptr = self._coords.ctypes.data
        self._h = lib().oxy_sim_create(n, self.m, edges, colour, cptr, L, self.nT, self.T, seed)
        if not self._h:
            raise ValueError("oxy_sim_create failed")
        self.n_colours = lib().oxy_sim_n_colours(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oxy_sim_free(h)
            self._h = None

    def init_random(self):
        lib().oxy_sim_init_random(self._h)

    def set_state(self, xy, slot_of_T=None, sweep=0):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(self.nT, self.n, 2)
        perm = None
        if slot_of_T is not None:
            self._perm = np.ascontiguousarray(slot_of_T, dtype=np.int32)
            perm = self._perm.ctypes.data
        lib().oxy_sim_set_state(self._h, xy, perm, sweep)

    def get_state(self):
        xy = np.empty((self.nT, self.n, 2), dtype=np.float64)
        perm = np.empty(self.nT, dtype=np.int32)
        sw = ctypes.c_uint32(0)
        lib().oxy_sim_get_state(self._h, xy, perm, ctypes.byref(sw))
        return xy, perm, sw.value

    def energy(self, slot):
        return lib().oxy_sim_energy(self._h, slot)

    def measure(self):
        out = np.empty((self.nT, NOBS), dtype=np.float64)
        lib().oxy_sim_measure(self._h, out)
        return out

    def run(self, n_sweeps, n_or=5, pt_every=0, meas_every=1, max_rec=None,
            met_log=False, pt_log=False):
        """Returns dict(records[n_rec, nT, 8], met_log[n_sweeps, nT, n], pt_log[n_sweeps, nT])."""
        if max_rec is None:
            max_rec = n_sweeps // meas_every if meas_every > 0 else 0
        rec = np.zeros((max(max_rec, 1), self.nT, NOBS), dtype=np.float64)
        ml = np.zeros((n_sweeps, self.nT, self.n), dtype=np.uint8) if met_log else None
        pl = np.zeros((n_sweeps, self.nT), dtype=np.uint8) if pt_log else None
        nrec = lib().oxy_sim_run(self._h, n_sweeps, n_or, pt_every, meas_every,
                                 rec.ctypes.data, max_rec,
                                 ml.ctypes.data if ml is not None else None,
                                 pl.ctypes.data if pl is not None else None)
        return {"records": rec[:nrec], "met_log": ml, "pt_log": pl}

    def pt_counts(self):
        acc = np.zeros(self.nT, dtype=np.int64)
        tries = np.zeros(self.nT, dtype=np.int64)
        lib().oxy_sim_pt_counts(self._h, acc, tries)
        return acc, tries
