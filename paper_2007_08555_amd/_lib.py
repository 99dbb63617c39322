"""ctypes declarations of libmtp's C ABI (include/mtp.h), nothing else.

The shared library is built in-tree by paper_2007_08555_amd.build; if it is
missing it is built on first use.  There is no fallback: every computation
runs in the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmtp.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "mtp.h")

MTP_FP64, MTP_FP32, MTP_FP32_COMPENSATED, MTP_MIXED = 0, 1, 2, 3
PRECISIONS = {"fp64": MTP_FP64, "fp32": MTP_FP32, "fp32c": MTP_FP32_COMPENSATED, "mixed": MTP_MIXED}
MTP_SCALE_MOLECULES, MTP_SCALE_STRUCTURES, MTP_SCALE_VIBRATIONS = 0, 1, 2
SCALINGS = {"molecules": 0, "structures": 1, "vibrations": 2}
ERRORS = {0: "MTP_OK", -1: "MTP_E_ARG", -2: "MTP_E_FILE", -3: "MTP_E_HIP",
          -4: "MTP_E_CAPACITY", -5: "MTP_E_BASIS", -6: "MTP_E_STATE"}


class mtp_batch(ctypes.Structure):
    _fields_ = [("n_configs", ctypes.c_int32), ("n_atoms", ctypes.c_int64),
                ("atom_offsets", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("species", ctypes.c_void_p), ("cell", ctypes.c_void_p), ("pbc", ctypes.c_void_p)]


class mtp_out(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_void_p), ("forces", ctypes.c_void_p), ("virial", ctypes.c_void_p),
                ("site_energy", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class mtp_info(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("m", ctypes.c_int32), ("n_mu", ctypes.c_int32),
                ("n_species", ctypes.c_int32), ("n_q", ctypes.c_int32), ("n_c", ctypes.c_int32),
                ("r_min", ctypes.c_double), ("r_cut", ctypes.c_double), ("n_schedules", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class mtp_stats(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("max_neighbours", ctypes.c_int32),
                ("level", ctypes.c_int32), ("flops_pair_fwd", ctypes.c_double), ("flops_pair_bwd", ctypes.c_double),
                ("flops_atom", ctypes.c_double), ("ms_neighbours", ctypes.c_float), ("ms_eval", ctypes.c_float),
                ("ms_forces", ctypes.c_float), ("ms_reduce", ctypes.c_float), ("lists_reused", ctypes.c_int32),
                ("list_builds", ctypes.c_int32)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "mtp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(_P)]),
    "mtp_model_info": (ctypes.c_int, [_P, ctypes.POINTER(mtp_info)]),
    "mtp_set_params": (ctypes.c_int, [_P, _P, _P]),
    "mtp_get_params": (ctypes.c_int, [_P, _P, _P]),
    "mtp_eval": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), ctypes.POINTER(mtp_out), ctypes.c_int, _P]),
    "mtp_eval_async": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), ctypes.POINTER(mtp_out), ctypes.c_int, _P]),
    "mtp_set_active_set": (ctypes.c_int, [_P, _P, _P]),
    "mtp_grade_from_b": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "mtp_grade_from_b_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "mtp_grade": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), _P, _P, ctypes.c_int, _P]),
    "mtp_theta_rows": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), ctypes.c_int, _P, _P]),
    "mtp_set_active_set_theta": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "mtp_grade_theta": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "mtp_kinetic_energy": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "mtp_fire_step": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "mtp_maxvol_theta": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P]),
    "mtp_status": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "mtp_loss_grad": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
    "mtp_normal_equations": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), _P, _P, _P, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, _P, _P, _P, _P]),
    "mtp_solve_normal": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "mtp_set_schedule": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "mtp_autotune": (ctypes.c_int, [_P, ctypes.POINTER(mtp_batch), ctypes.c_int, ctypes.c_int, _P, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), _P]),
    "mtp_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "mtp_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(mtp_stats)]),
    "mtp_set_skin": (ctypes.c_int, [_P, ctypes.c_double]),
    "mtp_md_kick": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_int, _P]),
    "mtp_maxvol": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32), _P]),
    "mtp_free": (None, [_P]),
    "mtp_last_error": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


def header_functions():
    """Names of the functions declared in include/mtp.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtp_[a-z_]+)\s*\(", text)))


def lib():
    """The loaded library (built first if it does not exist)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build
                build.build()
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


class MTPError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().mtp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(code, where):
    if code != 0:
        raise MTPError(code, where)
