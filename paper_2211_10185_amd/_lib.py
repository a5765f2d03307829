"""ctypes binding of ``libqfdtd.so`` (the C ABI declared in ``include/qfdtd.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqfdtd.so")

OK = 0
E_INVALID = -1
E_UNSUPPORTED_N = -2
E_UNSTABLE_DT = -3
E_NOMEM = -4
E_DEVICE = -5
E_NUMERIC = -6
E_STATE = -7
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_UNSUPPORTED_N", -3: "E_UNSTABLE_DT",
                -4: "E_NOMEM", -5: "E_DEVICE", -6: "E_NUMERIC", -7: "E_STATE"}

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class Potential(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("p", ct.c_double * 4), ("knots", ct.POINTER(ct.c_double)),
                ("n_knots", ct.c_int32), ("grid", ct.POINTER(ct.c_double))]


class Options(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("n_states", ct.c_int32),
                ("sectors", ct.POINTER(ct.c_int32)), ("measure_every", ct.c_int32),
                ("trace_energies", ct.c_int32), ("hip_stream", ct.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", ct.c_void_p),
                ("flags", ct.c_uint32)]

F_SINGLE_STREAM = 1
F_ROWCOL = 2
F_NO_GRAPH = 4
F_AB_SCHEME = 8
F_THREE_GROUPS = 16
F_STENCIL_1STEP = 32
F_SPLIT_X2 = 64
F_SPLIT_NARROW = 128
F_SPLIT_WIDE = 256
F_SPLIT_SWAPPED = 384


class QfdtdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError("libqfdtd.so is not built: run `python -m paper_2211_10185_amd.build` "
                      "(expected at %s)" % LIB_PATH)

# PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Load it first so that the library binds to that one runtime; loading the
# library first would bring in a second runtime that cannot see the device.
import torch  # noqa: E402,F401

lib = ct.CDLL(LIB_PATH)

P = ct.c_void_p
DP = ct.POINTER(ct.c_double)
_sig = {
    "qfdtd_create": (ct.c_int, [ct.POINTER(P), ct.c_int32, ct.c_double, ct.c_double, ct.c_int32,
                                ct.POINTER(Potential), ct.POINTER(Options)]),
    "qfdtd_set_state": (ct.c_int, [P, ct.c_int32, DP]),
    "qfdtd_set_state_device": (ct.c_int, [P, ct.c_int32, P]),
    "qfdtd_set_state_noise": (ct.c_int, [P, ct.c_int32, ct.c_uint64]),
    "qfdtd_evolve": (ct.c_int, [P, ct.c_int64, ct.c_double]),
    "qfdtd_states": (ct.c_int, [P, ct.c_int32, DP, DP]),
    "qfdtd_states_device": (ct.c_int, [P, ct.c_int32, DP, P]),
    "qfdtd_energy_trace": (ct.c_int, [P, DP, ct.c_int64, ct.POINTER(ct.c_int64)]),
    "qfdtd_batch_evolve": (ct.c_int, [ct.POINTER(P), ct.c_int32, ct.POINTER(ct.c_int64), DP]),
    "qfdtd_batch_energies": (ct.c_int, [ct.POINTER(P), ct.c_int32, DP]),
    "qfdtd_gram_matrix": (ct.c_int, [P, DP]),
    "qfdtd_gram_residuals": (ct.c_int, [P, DP]),
    "qfdtd_gram_matrix_noalloc": (ct.c_int, [P, ct.c_int64, ct.c_int32, ct.c_int32, P, P]),
    "qfdtd_read_potential_ascii": (ct.c_int, [ct.c_char_p, ct.c_int32, DP]),
    "qfdtd_write_potential_ascii": (ct.c_int, [ct.c_char_p, ct.c_int32, DP]),
    "qfdtd_footprint": (ct.c_size_t, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32]),
    "qfdtd_enable_kernel_timing": (ct.c_int, [P, ct.c_int32]),
    "qfdtd_kernel_stats": (ct.c_int, [P, ct.c_int32, ct.POINTER(ct.c_int64), DP, DP]),
    "qfdtd_transform_state": (ct.c_int, [P, ct.c_int32, ct.c_int32]),
    "qfdtd_state_pointer": (ct.c_int, [P, ct.c_int32, ct.POINTER(P)]),
    "qfdtd_destroy": (None, [P]),
    "qfdtd_last_error": (ct.c_char_p, [P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def check(status, ctx=None):
    if status != OK:
        msg = lib.qfdtd_last_error(ctx)
        raise QfdtdError(status, msg.decode() if msg else "")
    return status


def exported_symbols():
    return sorted(_sig)
