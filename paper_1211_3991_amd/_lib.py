"""ctypes binding of libxylevy.so (include/xy_levy.h): argument marshalling only.

Every step of the method runs inside the library: the host graph path in its
C++ code and the sweeps, tempering and measurements in its HIP kernels.  If
the library is missing this module raises at import; there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxylevy.so")

XY_OK, XY_EINVAL, XY_ENOMEM, XY_EHIP, XY_ESTATE, XY_EUNSUP, XY_ECONVERGE = 0, -1, -2, -3, -4, -5, -6
XY_FP64, XY_FIX16 = 0, 1
XY_NOBS = 8
STATUS_NAMES = {0: "XY_OK", -1: "XY_EINVAL", -2: "XY_ENOMEM", -3: "XY_EHIP", -4: "XY_ESTATE",
                -5: "XY_EUNSUP", -6: "XY_ECONVERGE"}

EXPORTS = ("xy_graph_levy", "xy_graph_levy_free", "xy_graph_from_edges", "xy_graph_info", "xy_graph_export", "xy_graph_free",
           "xy_batch_sizes", "xy_batch_init", "xy_sweep", "xy_measure", "xy_pt_energies", "xy_pt_swap", "xy_get_state",
           "xy_set_state", "xy_get_counters", "xy_decision_log", "xy_batch_use_graph", "xy_batch_set_fix16_form", "xy_batch_set_phase_streams", "xy_batch_phase_streams", "xy_batch_set_phase_groups", "xy_batch_phase_groups", "xy_batch_forms", "xy_walk_bytes", "xy_random_walk", "xy_random_walk_noalloc", "xy_kernel_timing",
           "xy_kernel_time", "xy_last_error", "xy_batch_free")


class XYError(RuntimeError):
    def __init__(self, status, what, msg):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Sizes(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_size_t), ("graph_bytes", ctypes.c_size_t),
                ("work_bytes", ctypes.c_size_t), ("obs_bytes", ctypes.c_size_t)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(the HIP library is required, there is no fallback)")

# PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
# first makes the library's libamdhip64.so.7 dependency resolve to that same,
# already loaded runtime, so device pointers and streams handed over by torch
# belong to the runtime the library calls.  Loading the library first would
# bring in a second HIP runtime from the system ROCm.
import torch  # noqa: E402,F401

_c = ctypes.CDLL(LIB_PATH)
_vp, _i32, _u32, _u64, _dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_sigs = {
    "xy_graph_levy": ([_i32, _i32, _dbl, _u64, ctypes.POINTER(_vp)], _i32),
    "xy_graph_levy_free": ([_i32, _i32, _dbl, _u64, ctypes.POINTER(_vp)], _i32),
    "xy_graph_from_edges": ([_i32, _i32, _vp, _vp, _i32, ctypes.POINTER(_vp)], _i32),
    "xy_graph_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                       ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_int64)], _i32),
    "xy_graph_export": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "xy_graph_free": ([_vp], None),
    "xy_batch_sizes": ([_vp, _i32, _i32, _i32, _i32, ctypes.POINTER(Sizes)], _i32),
    "xy_batch_init": ([ctypes.POINTER(_vp), _vp, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "xy_sweep": ([_vp, _vp, _i32, _i32, _i32, _i32, _vp], _i32),
    "xy_measure": ([_vp, _vp, _vp], _i32),
    "xy_pt_energies": ([_vp, _vp, _vp], _i32),
    "xy_pt_swap": ([_vp, _vp], _i32),
    "xy_get_state": ([_vp, _vp, _vp, ctypes.POINTER(_u32), _vp], _i32),
    "xy_set_state": ([_vp, _vp, _vp, _u32, _vp], _i32),
    "xy_get_counters": ([_vp, ctypes.POINTER(_i32), _vp, _vp, _vp], _i32),
    "xy_decision_log": ([_vp, _vp, _i32], _i32),
    "xy_batch_use_graph": ([_vp, _i32], _i32),
    "xy_batch_set_fix16_form": ([_vp, _i32, _i32, _i32, _vp], _i32),
    "xy_batch_forms": ([_vp, _vp], _i32),
    "xy_batch_set_phase_streams": ([_vp, _i32, _vp], _i32),
    "xy_batch_phase_streams": ([_vp, _vp], _i32),
    "xy_batch_set_phase_groups": ([_vp, _i32, _i32, _vp], _i32),
    "xy_batch_phase_groups": ([_vp, _vp, _vp], _i32),
    "xy_walk_bytes": ([_vp, _i32, ctypes.POINTER(ctypes.c_size_t)], _i32),
    "xy_random_walk": ([_vp, _i32, _i32, _i32, _vp, _i32, _vp, ctypes.c_size_t, _vp, _vp,
                        ctypes.POINTER(ctypes.c_float)], _i32),
    "xy_random_walk_noalloc": ([_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_float)], _i32),
    "xy_kernel_timing": ([_vp, _i32], _i32),
    "xy_kernel_time": ([_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_i32)], _i32),
    "xy_last_error": ([], ctypes.c_char_p),
    "xy_batch_free": ([_vp], None),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_c, _name)
    _f.argtypes = _args
    _f.restype = _res


def call(name, *args):
    """Calls an xy_* entry point and raises XYError on a non-zero status."""
    st = getattr(_c, name)(*args)
    if st != XY_OK:
        raise XYError(st, name, _c.xy_last_error().decode(errors="replace"))
    return st


def raw():
    return _c
