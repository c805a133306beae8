"""ctypes binding of libtgms.so (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
tensors to device pointers and status codes to exceptions.  It raises if the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtgms.so")

c_int, c_double, c_void_p, c_char_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p

STATUS = {0: "OK", -1: "INVAL", -2: "INCOMPAT", -3: "NOTCONV", -4: "BREAKDOWN", -5: "DEVICE", -6: "NOMEM",
          -7: "UNSUPPORTED"}


class TgmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tgms {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("nx", c_int), ("ny", c_int), ("nz", c_int), ("bx", c_int), ("by", c_int),
                ("bz", c_int)]


class Options(ctypes.Structure):
    _fields_ = [("eta", c_double), ("overlap", c_int), ("precision", c_int), ("s_scale", c_double),
                ("stream", c_void_p), ("graphs", c_int), ("autotune", c_int), ("tune_cache", c_char_p),
                ("warm_start", c_int), ("cnn_weights", c_void_p), ("rq_tol", c_double),
                ("smoother_staging", c_int), ("rows_per_thread", c_int), ("force_counts", c_void_p),
                ("coarse_space", c_int), ("coarse_factor", c_int), ("smooth_steps", c_int), ("additive", c_int)]


class Info(ctypes.Structure):
    _fields_ = [("n_coarse_faces", c_int), ("n_blocks", c_int), ("dim", c_int), ("n_coarse_spd", c_int),
                ("t_setup_ms", c_double), ("t_snap_ms", c_double), ("t_eig_ms", c_double),
                ("t_coarse_ms", c_double), ("t_smoother_ms", c_double), ("lds_max", c_int), ("pcg_graph", c_int),
                ("tuned", c_int), ("nred", c_int), ("smooth_staged", c_int), ("warm_accepted", c_int),
                ("warm_iters", c_int), ("t_cnn_ms", c_double), ("rows_per_thread", c_int),
                ("eig_unconverged", c_int), ("coarse_space", c_int), ("nx", c_int), ("ny", c_int), ("bx", c_int),
                ("by", c_int), ("precision", c_int), ("coarse_block", c_int), ("rt0_block", c_int)]


class TransportParams(ctypes.Structure):
    _fields_ = [("phi", c_double), ("mu_w", c_double), ("mu_o", c_double), ("tol", c_double),
                ("max_outer", c_int)]


_lib = None

# name -> (restype, argtypes); the exported C ABI of include/tgms.h
SIGNATURES = {
    "tgms_default_options": (None, [ctypes.POINTER(Options)]),
    "tgms_setup": (c_int, [ctypes.POINTER(Grid), c_void_p, c_double, ctypes.POINTER(Options), ctypes.POINTER(c_void_p)]),
    "tgms_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p, c_void_p,
                           ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
    "tgms_solve_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p, c_void_p,
                                   ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
    "tgms_info": (c_int, [c_void_p, ctypes.POINTER(Info)]),
    "tgms_get_counts": (c_int, [c_void_p, c_void_p]),
    "tgms_get_eigs": (c_int, [c_void_p, c_void_p]),
    "tgms_last_cond": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "tgms_profile": (c_int, [c_void_p, c_int]),
    "tgms_profile_get": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double)]),
    "tgms_time_smoother": (c_int, [c_void_p, c_int, ctypes.POINTER(c_double)]),
    "tgms_time_dir_apply": (c_int, [c_void_p, c_int, ctypes.POINTER(c_double)]),
    "tgms_destroy": (None, [c_void_p]),
    "tgms_last_error": (c_char_p, []),
    "tgms_apply_A": (c_int, [c_void_p, c_void_p, c_void_p]),
    "tgms_preprocess": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "tgms_apply_precond": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "tgms_update_mobility": (c_int, [c_void_p, c_void_p]),
    "tgms_get_warm_status": (c_int, [c_void_p, c_void_p]),
    "tgms_cnn_nparams": (c_int, []),
    "tgms_cnn_forward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p]),
    "tgms_cnn_infer": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p]),
    "tgms_cnn_train_workspace": (ctypes.c_size_t, [c_int, c_int, c_int]),
    "tgms_cnn_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float, c_void_p, c_void_p, c_int,
                                    c_int, c_int, c_int, c_void_p, ctypes.POINTER(c_double), c_void_p]),
    "tgms_cnn_samples": (c_int, [c_void_p, c_void_p, c_void_p]),
    "tgms_save": (c_int, [c_void_p, c_char_p]),
    "tgms_load": (c_int, [c_char_p, ctypes.POINTER(Options), ctypes.POINTER(c_void_p)]),
    "tgms_probe_pencil": (c_int, [c_void_p, c_void_p, c_void_p]),
    "tgms_trim_device_cache": (None, []),
    "tgms_default_transport": (None, [ctypes.POINTER(TransportParams)]),
    "tgms_total_mobility": (c_int, [c_void_p, ctypes.c_longlong, ctypes.POINTER(TransportParams), c_void_p,
                                    c_void_p]),
    "tgms_transport_step": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_double,
                                    ctypes.POINTER(TransportParams), c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(c_double)]),
    "tgms_impes": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, c_int, ctypes.POINTER(TransportParams),
                           c_double, c_int, c_void_p, c_void_p]),
}


def load():
    """Load libtgms.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1807_07220_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code):
    if code != 0:
        raise TgmsError(code, load().tgms_last_error().decode())
