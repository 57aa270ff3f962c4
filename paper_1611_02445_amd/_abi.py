"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only).

The shared library is built in-tree by ``paper_1611_02445_amd.build``; if it is
missing this module raises instead of falling back to anything else.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtiledlbm.so")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_E_INVAL", -2: "LBM_E_NOMEM", -3: "LBM_E_RANGE", -4: "LBM_E_HIP",
          -5: "LBM_E_STATE", -6: "LBM_E_UNSUPPORTED", -7: "LBM_E_NUMERIC"}
STATUS_CODE = {name: code for code, name in STATUS.items()}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2}
MODEL = {"qc": 0, "quasi-compressible": 0, "inc": 1, "incompressible": 1, "mrt-qc": 2, "mrt-inc": 3}

# every symbol include/lbm.h declares
EXPORTS = [
    "lbm_build_tiles", "lbm_tiles_free", "lbm_tile_order", "lbm_required_bytes", "lbm_create", "lbm_destroy", "lbm_init",
    "lbm_set_force", "lbm_set_boundaries", "lbm_step", "lbm_step_graphed", "lbm_step_buf", "lbm_current_state", "lbm_macroscopic", "lbm_macroscopic_buf",
    "lbm_macroscopic_noalloc",
    "lbm_permeability", "lbm_get_state", "lbm_set_state", "lbm_tiles_to_dense", "lbm_field_to_dense",
    "lbm_adjoint_seed",
    "lbm_adjoint_step", "lbm_adjoint_final", "lbm_adjoint_get", "lbm_adjoint_set", "lbm_calib_step",
    "lbm_stream_probe", "lbm_info",
    "lbm_last_error", "lbm_version",
]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Tiles(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tx", ctypes.c_int32), ("ty", ctypes.c_int32), ("tz", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("n_fluid", ctypes.c_int64),
                ("eta_t", ctypes.c_double),
                ("tile_map", ctypes.POINTER(ctypes.c_int32)), ("tile_xyz", ctypes.POINTER(ctypes.c_int32)),
                ("nbr", ctypes.POINTER(ctypes.c_int32)), ("fluid_mask", ctypes.POINTER(ctypes.c_uint64))]


class Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("rho0", ctypes.c_double), ("storage", ctypes.c_int32),
                ("model", ctypes.c_int32), ("f16_log2_scale", ctypes.c_int32), ("tiles_per_wg", ctypes.c_int32),
                ("f16_rounding", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("wide_offsets", ctypes.c_int32), ("f32_unshifted", ctypes.c_int32),
                ("check_u_max", ctypes.c_int32)]


class Sizes(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_size_t), ("table_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t), ("force_bytes", ctypes.c_size_t),
                ("adjoint_bytes", ctypes.c_size_t), ("grad_force_bytes", ctypes.c_size_t),
                ("bc_bytes", ctypes.c_size_t), ("dense_nodes", ctypes.c_size_t)]


_lib = None


def lib():
    """Load libtiledlbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1611_02445_amd.build` "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    TP = ctypes.POINTER(Tiles)
    sig = {
        "lbm_build_tiles": ([P, i32, i32, i32, i32, ctypes.POINTER(TP)], ctypes.c_int),
        "lbm_tiles_free": ([TP], None),
        "lbm_tile_order": ([TP, i32, P], ctypes.c_int),
        "lbm_required_bytes": ([TP, ctypes.POINTER(Params), ctypes.POINTER(Sizes)], ctypes.c_int),
        "lbm_create": ([TP, ctypes.POINTER(Params), P, P, P, P, P, ctypes.POINTER(P)], ctypes.c_int),
        "lbm_destroy": ([P], ctypes.c_int),
        "lbm_init": ([P, f64, f64, f64, f64], ctypes.c_int),
        "lbm_set_force": ([P, f64, f64, f64, P, P], ctypes.c_int),
        "lbm_set_boundaries": ([P, P, f64, f64, f64, f64, P], ctypes.c_int),
        "lbm_step": ([P, i32], ctypes.c_int),
        "lbm_step_graphed": ([P, i32], ctypes.c_int),
        "lbm_step_buf": ([P, P, P], ctypes.c_int),
        "lbm_current_state": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "lbm_macroscopic": ([P, P, P, P], ctypes.c_int),
        "lbm_macroscopic_buf": ([P, P, P, P, P], ctypes.c_int),
        "lbm_macroscopic_noalloc": ([P, P, P, P, P], ctypes.c_int),
        "lbm_permeability": ([P, f64, ctypes.POINTER(f64)], ctypes.c_int),
        "lbm_get_state": ([P, P, P], ctypes.c_int),
        "lbm_set_state": ([P, P, P], ctypes.c_int),
        "lbm_tiles_to_dense": ([P, P, i32, i32, P], ctypes.c_int),
        "lbm_field_to_dense": ([P, P, i32, P], ctypes.c_int),
        "lbm_adjoint_seed": ([P, P, P, P], ctypes.c_int),
        "lbm_adjoint_step": ([P, P, P, P, P], ctypes.c_int),
        "lbm_adjoint_final": ([P, P, P], ctypes.c_int),
        "lbm_adjoint_get": ([P, P, P], ctypes.c_int),
        "lbm_adjoint_set": ([P, P, P], ctypes.c_int),
        "lbm_calib_step": ([P, i32, P, P], ctypes.c_int),
        "lbm_stream_probe": ([P, i32, P, P, ctypes.c_size_t, i32, i32], ctypes.c_int),
        "lbm_info": ([P, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)],
                     ctypes.c_int),
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


def call(name, *args):
    return check(getattr(lib(), name)(*args))
