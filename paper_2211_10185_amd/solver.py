"""Python front end of the HIP solver: one ``Solver`` per lattice problem.

The solver state lives on the GPU for its whole life.  Device memory comes from
PyTorch's caching allocator (through the C ABI's allocator hook) and work is
ordered on PyTorch's current HIP stream; PyTorch does nothing else here.
"""
from __future__ import annotations

import ctypes as ct
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

FDTD, NR_P2, NR_SIN2, REL = 0, 1, 2, 3
V_GRID, V_HARMONIC, V_CORNELL, V_COULOMB, V_RADIAL_SPLINE = 0, 1, 2, 3, 4
C64, C128 = 0, 1

CLASS_PLANE, CLASS_ROW, CLASS_COL, CLASS_STENCIL = 0, 1, 2, 3


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to PyTorch")
    return torch


class _TorchAllocator:
    """C-callable allocate/free pair backed by torch's caching allocator."""

    def __init__(self, stream_ptr):
        torch = _torch()
        self._torch = torch
        dev = torch.cuda.current_device()
        self._dev = dev
        self._stream = stream_ptr   # a torch.cuda.Stream

        def _alloc(nbytes, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, self._stream))
            except Exception:
                return None

        def _free(ptr, user):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = L.ALLOC_FN(_alloc)
        self.free = L.FREE_FN(_free)


def potential_struct(kind: int, params: Sequence[float] = (), knots: Optional[np.ndarray] = None,
                     grid: Optional[np.ndarray] = None):
    """Build the C potential description; returns (struct, keepalive arrays)."""
    pot = L.Potential()
    pot.kind = int(kind)
    for i, v in enumerate(list(params)[:4]):
        pot.p[i] = float(v)
    keep = []
    if knots is not None:
        kn = np.ascontiguousarray(np.asarray(knots, dtype=np.float64).reshape(-1, 2))
        keep.append(kn)
        pot.knots = kn.ctypes.data_as(ct.POINTER(ct.c_double))
        pot.n_knots = kn.shape[0]
    if grid is not None:
        g = np.ascontiguousarray(np.asarray(grid, dtype=np.complex128))
        keep.append(g)
        pot.grid = g.ctypes.data_as(ct.POINTER(ct.c_double))
    return pot, keep


class Solver:
    """Imaginary-time solver for k states on an N^3 lattice (C ABI ``qfdtd_*``)."""

    def __init__(self, N: int, a: float, m: float, kinetic: int, vkind: int,
                 vparams: Sequence[float] = (), knots=None, grid=None, precision: int = C64,
                 n_states: int = 3, sectors: Optional[Sequence[int]] = None,
                 measure_every: int = 50, trace: bool = False, torch_alloc: bool = True,
                 single_stream: Optional[bool] = None, rowcol: Optional[bool] = None,
                 graphs: bool = True, scheme: int = 0, groups: Optional[int] = None,
                 fused_stencil: bool = True, split: Optional[bool] = None,
                 split_variant: Optional[int] = None):
        torch = _torch()
        self.N, self.a, self.m, self.kinetic = int(N), float(a), float(m), int(kinetic)
        self.precision, self.k = int(precision), int(n_states)
        self.stream = torch.cuda.current_stream()
        self._alloc = _TorchAllocator(self.stream) if torch_alloc else None
        pot, self._keep = potential_struct(vkind, vparams, knots, grid)
        opt = L.Options()
        opt.precision = self.precision
        opt.n_states = self.k
        if sectors is not None:
            sec = (ct.c_int32 * self.k)(*[int(s) for s in sectors])
            self._keep.append(sec)
            opt.sectors = ct.cast(sec, ct.POINTER(ct.c_int32))
        opt.measure_every = int(measure_every)
        opt.trace_energies = 1 if trace else 0
        # state groups on their own streams (FFT plane schedule): 1, 2 or 3
        if groups is not None:
            single_stream = int(groups) <= 1
        if single_stream is None or rowcol is None or groups is None or split is None:
            from .autotune import schedule_for
            tuned = schedule_for(self.N, self.kinetic, self.precision, self.k)
            single_stream = tuned["single_stream"] if single_stream is None else single_stream
            rowcol = tuned["rowcol"] if rowcol is None else rowcol
            if split is None:
                split = tuned.get("split", False)
                if split_variant is None:
                    split_variant = int(tuned.get("split_variant", 0))
            if groups is None:
                groups = 1 if single_stream else int(tuned.get("groups", 2))
        split_variant = int(split_variant or 0)
        self.schedule = {"single_stream": bool(single_stream), "rowcol": bool(rowcol), "groups": int(groups),
                         "split": bool(split), "split_variant": split_variant}
        # scheme 1: the A/B update (psi' = A psi - B dt H_K psi) for the FFT kinetic terms
        self.scheme = int(scheme)
        opt.flags = ((L.F_SINGLE_STREAM if single_stream else 0) | (L.F_ROWCOL if rowcol else 0)
                     | (0 if graphs else L.F_NO_GRAPH) | (L.F_AB_SCHEME if self.scheme == 1 else 0)
                     | (L.F_THREE_GROUPS if int(groups) == 3 else 0)
                     | (0 if fused_stencil else L.F_STENCIL_1STEP) | (L.F_SPLIT_X2 if split else 0)
                     | ((split_variant & 3) << 7 if split else 0))
        opt.hip_stream = ct.c_void_p(self.stream.cuda_stream)
        if self._alloc is not None:
            opt.dev_alloc = self._alloc.alloc
            opt.dev_free = self._alloc.free
        self._ctx = ct.c_void_p()
        L.check(L.lib.qfdtd_create(ct.byref(self._ctx), self.N, self.a, self.m, self.kinetic,
                                   ct.byref(pot), ct.byref(opt)))
        self._keep = None

    @classmethod
    def from_problem(cls, p, precision: Optional[int] = None, trace: bool = False, **kw):
        """Build from a ``synthetic.Problem`` (potential evaluated on the device)."""
        grid = p.abi_grid()
        s = cls(p.N, p.a, p.m, p.kinetic, p.vkind, p.vparams, knots=p.knots, grid=grid,
                precision=p.precision if precision is None else precision, n_states=p.k,
                sectors=p.sectors, measure_every=p.measure_every, trace=trace,
                **dict({"scheme": getattr(p, "scheme", 0)}, **kw))
        return s

    @property
    def ctx(self):
        return self._ctx

    def _c(self, status):
        return L.check(status, self._ctx)

    def set_state(self, i: int, psi: np.ndarray):
        a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).reshape(-1)
        if a.size != self.N ** 3:
            raise ValueError("state must have N^3 elements")
        self._c(L.lib.qfdtd_set_state(self._ctx, int(i), a.ctypes.data_as(ct.POINTER(ct.c_double))))

    def set_states(self, psis: np.ndarray):
        for i in range(self.k):
            self.set_state(i, psis[i])

    def set_states_noise(self, seed: int):
        """Every state from the library's seeded device noise (stream-ordered, no host array)."""
        for i in range(self.k):
            self._c(L.lib.qfdtd_set_state_noise(self._ctx, i, int(seed) & 0xFFFFFFFFFFFFFFFF))

    def evolve(self, steps: int, dt: float):
        self._c(L.lib.qfdtd_evolve(self._ctx, int(steps), float(dt)))

    def states(self, k: Optional[int] = None, with_psi: bool = True):
        k = self.k if k is None else int(k)
        e = np.zeros(2 * k, dtype=np.float64)
        psi = np.zeros((k, self.N, self.N, self.N), dtype=np.complex128) if with_psi else None
        pp = psi.ctypes.data_as(ct.POINTER(ct.c_double)) if with_psi else None
        self._c(L.lib.qfdtd_states(self._ctx, k, e.ctypes.data_as(ct.POINTER(ct.c_double)), pp))
        E = e[0::2] + 1j * e[1::2]
        return (E, psi) if with_psi else E

    def energies(self):
        return self.states(with_psi=False)

    def gram(self) -> np.ndarray:
        """FP64 Gram matrix <psi_i|psi_j> of the current states (k x k, complex)."""
        g = np.zeros(2 * self.k * self.k, dtype=np.float64)
        self._c(L.lib.qfdtd_gram_matrix(self._ctx, g.ctypes.data_as(ct.POINTER(ct.c_double))))
        return (g[0::2] + 1j * g[1::2]).reshape(self.k, self.k)

    def residuals(self) -> np.ndarray:
        """Norm of each state after projection against the earlier states of its sector (the
        diagonal of the device FP64 Cholesky factor of the Gram matrix)."""
        r = np.zeros(self.k, dtype=np.float64)
        self._c(L.lib.qfdtd_gram_residuals(self._ctx, r.ctypes.data_as(ct.POINTER(ct.c_double))))
        return r

    def set_state_device(self, i: int, t):
        """State i from a contiguous device tensor in the solver's precision (stream-ordered)."""
        torch = _torch()
        want = torch.complex64 if self.precision == C64 else torch.complex128
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.numel() != self.N ** 3:
            raise ValueError("need a contiguous CUDA tensor of N^3 %s elements" % want)
        self._c(L.lib.qfdtd_set_state_device(self._ctx, int(i), ct.c_void_p(t.data_ptr())))

    def energy_trace(self):
        n = ct.c_int64()
        self._c(L.lib.qfdtd_energy_trace(self._ctx, None, 0, ct.byref(n)))
        out = np.zeros((max(n.value, 1), self.k, 2))
        self._c(L.lib.qfdtd_energy_trace(self._ctx, out.ctypes.data_as(ct.POINTER(ct.c_double)),
                                         n.value, ct.byref(n)))
        t = out[: n.value]
        return t[..., 0] + 1j * t[..., 1]

    def transform_state(self, i: int, sign: int):
        self._c(L.lib.qfdtd_transform_state(self._ctx, int(i), int(sign)))

    def state_tensor(self, i: int):
        """Device view of state i as a torch complex tensor (shares memory)."""
        torch = _torch()
        p = ct.c_void_p()
        self._c(L.lib.qfdtd_state_pointer(self._ctx, int(i), ct.byref(p)))
        dtype = torch.complex64 if self.precision == C64 else torch.complex128
        n = self.N ** 3
        # wrap the raw device pointer without copying
        class _Arr:
            __cuda_array_interface__ = {
                "shape": (n,), "typestr": "<c8" if self.precision == C64 else "<c16",
                "data": (p.value, False), "version": 3, "strides": None}
        return torch.as_tensor(_Arr(), device="cuda").view(self.N, self.N, self.N)

    def enable_kernel_timing(self, every: int = 1):
        self._c(L.lib.qfdtd_enable_kernel_timing(self._ctx, int(every)))

    def kernel_stats(self, cls: int):
        n = ct.c_int64()
        ms = ct.c_double()
        b = ct.c_double()
        self._c(L.lib.qfdtd_kernel_stats(self._ctx, int(cls), ct.byref(n), ct.byref(ms), ct.byref(b)))
        return n.value, ms.value, b.value

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            L.lib.qfdtd_destroy(self._ctx)
            self._ctx = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_evolve(solvers: Sequence[Solver], steps, dt):
    n = len(solvers)
    arr = (ct.c_void_p * n)(*[s.ctx.value for s in solvers])
    st = (ct.c_int64 * n)(*([int(steps)] * n if np.isscalar(steps) else [int(x) for x in steps]))
    d = (ct.c_double * n)(*([float(dt)] * n if np.isscalar(dt) else [float(x) for x in dt]))
    L.check(L.lib.qfdtd_batch_evolve(arr, n, st, d))


def batch_energies(solvers: Sequence[Solver]):
    n = len(solvers)
    kmax = max(s.k for s in solvers)
    arr = (ct.c_void_p * n)(*[s.ctx.value for s in solvers])
    e = np.zeros(2 * n * kmax)
    L.check(L.lib.qfdtd_batch_energies(arr, n, e.ctypes.data_as(ct.POINTER(ct.c_double))))
    e = e.reshape(n, kmax, 2)
    return e[..., 0] + 1j * e[..., 1]


def footprint(N: int, kinetic: int, precision: int, n_states: int) -> int:
    return int(L.lib.qfdtd_footprint(int(N), int(kinetic), int(precision), int(n_states)))


def read_potential_file(path: str, N: int) -> np.ndarray:
    """Complex potential grid [N, N, N] from an ASCII file (parsed by the library)."""
    g = np.zeros(2 * N ** 3, dtype=np.float64)
    L.check(L.lib.qfdtd_read_potential_ascii(str(path).encode(), int(N), g.ctypes.data_as(ct.POINTER(ct.c_double))),
            None)
    return (g[0::2] + 1j * g[1::2]).reshape(N, N, N)


def write_potential_file(path: str, grid: np.ndarray):
    """Write a complex grid [N, N, N] as an ASCII potential file (library writer)."""
    a = np.ascontiguousarray(np.asarray(grid, dtype=np.complex128))
    N = a.shape[0]
    L.check(L.lib.qfdtd_write_potential_ascii(str(path).encode(), int(N), a.view(np.float64).ctypes.data_as(
        ct.POINTER(ct.c_double))), None)
