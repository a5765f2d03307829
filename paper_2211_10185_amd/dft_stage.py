"""ctypes binding of ``libdftstage.so`` (``include/dft_stage.h``): a batched 16-point DFT stage
on the FP32 vector ALUs (the solver's radix-16 butterfly) and on FP32 MFMA (a dense 16 x 16
complex product), timed on the same data.

Argument marshalling only; importing raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdftstage.so")
VALU = 0
MFMA = 1
VARIANTS = {"valu": VALU, "mfma": MFMA}

if not os.path.exists(LIB_PATH):
    raise ImportError("libdftstage.so is not built: run `python -m paper_2211_10185_amd.build` "
                      "(expected at %s)" % LIB_PATH)

import torch  # noqa: E402  (load PyTorch's HIP runtime first, as for libqfdtd.so)

lib = ct.CDLL(LIB_PATH)
_P = ct.c_void_p
_sig = {
    "dft16_stage_run": (ct.c_int, [ct.c_int32, _P, _P, ct.c_int64, ct.c_int32, _P]),
    "dft16_stage_time": (ct.c_int, [ct.c_int32, _P, _P, ct.c_int64, ct.c_int32, ct.c_int32, _P,
                                    ct.POINTER(ct.c_double)]),
    "dft16_stage_last_error": (ct.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return sorted(_sig)


def _check(rc):
    if rc != 0:
        raise RuntimeError("dft16 stage: %d: %s" % (rc, lib.dft16_stage_last_error().decode()))


def _args(x, out):
    if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or x.shape[-1] != 16:
        raise ValueError("need a contiguous CUDA complex64 tensor of shape (nvec, 16)")
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must match x")
    nvec = x.numel() // 16
    if nvec % 256:
        raise ValueError("the number of vectors must be a multiple of 256")
    return nvec


def run(x, reps: int = 1, variant: str = "valu", out=None):
    """Apply the stage ``reps`` times (forward, inverse / 16, ...) to every row of ``x``."""
    out = torch.empty_like(x) if out is None else out
    nvec = _args(x, out)
    st = torch.cuda.current_stream().cuda_stream
    _check(lib.dft16_stage_run(VARIANTS[variant], x.data_ptr(), out.data_ptr(), nvec, int(reps), st))
    return out


def time_launch(x, out, reps: int, variant: str, iters: int = 20) -> float:
    """Mean milliseconds per launch over ``iters`` back-to-back launches (HIP events)."""
    nvec = _args(x, out)
    ms = ct.c_double()
    st = torch.cuda.current_stream().cuda_stream
    _check(lib.dft16_stage_time(VARIANTS[variant], x.data_ptr(), out.data_ptr(), nvec, int(reps), int(iters),
                                st, ct.byref(ms)))
    return ms.value
