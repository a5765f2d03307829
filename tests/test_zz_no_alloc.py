"""qfdtd_gram_matrix_noalloc (no context, no allocation) against qfdtd_gram_matrix."""
import ctypes as ct

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


def _gram_noalloc(ptr, n_sites, k, precision, stream):
    import torch
    from paper_2211_10185_amd import _lib as L
    G = torch.full((k, k, 2), float("nan"), dtype=torch.float64, device="cuda")
    st = L.lib.qfdtd_gram_matrix_noalloc(ct.c_void_p(ptr), n_sites, k, precision, ct.c_void_p(G.data_ptr()),
                                         ct.c_void_p(stream.cuda_stream))
    L.check(st)
    stream.synchronize()
    g = G.cpu().numpy()
    return g[..., 0] + 1j * g[..., 1]


@pytest.mark.parametrize("first,second", [((32, 3, 0), (16, 2, 1))])
def test_gram_without_allocation_matches_the_context_entry_point(first, second):
    from paper_2211_10185_amd import _lib as L
    from paper_2211_10185_amd.solver import Solver
    for N, k, prec in (first, second):       # two calls in a row, the second with a smaller input
        p = S.Problem(N=N, a=0.25, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,), k=k,
                      precision=prec, dt=0.01, steps=0, seed=40 + N)
        print("gram no-alloc: N", N, "k", k, "precision", prec, flush=True)
        s = Solver.from_problem(p)
        s.set_states(p.init_states())
        G_ctx = s.gram()
        ptr = ct.c_void_p()
        s._c(L.lib.qfdtd_state_pointer(s.ctx, 0, ct.byref(ptr)))
        G_na = _gram_noalloc(ptr.value, N ** 3, k, prec, s.stream)
        s.close()
        assert np.array_equal(G_na, G_ctx), (G_na, G_ctx)
        # against numpy on the same states (the solver's precision rounds them first)
        psi = p.init_states().reshape(k, -1)
        if prec == 0:
            psi = psi.astype(np.complex64).astype(np.complex128)
        np.testing.assert_allclose(G_na, psi.conj() @ psi.T, rtol=1e-12, atol=1e-9)


def test_gram_without_allocation_rejects_sizes_beyond_its_limit():
    import torch
    from paper_2211_10185_amd import _lib as L
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    G = torch.zeros(2 * 81, dtype=torch.float64, device="cuda")
    f = L.lib.qfdtd_gram_matrix_noalloc
    assert f(ct.c_void_p(buf.data_ptr()), 1, 9, 0, ct.c_void_p(G.data_ptr()), None) == L.E_INVALID
    assert f(ct.c_void_p(buf.data_ptr()), (1 << 27) + 1, 1, 0, ct.c_void_p(G.data_ptr()), None) == L.E_INVALID
    assert b"n_sites" in L.lib.qfdtd_last_error(None)
    assert f(ct.c_void_p(buf.data_ptr()), 0, 1, 0, ct.c_void_p(G.data_ptr()), None) == L.E_INVALID
    assert f(None, 1, 1, 0, ct.c_void_p(G.data_ptr()), None) == L.E_INVALID
    assert f(ct.c_void_p(buf.data_ptr()), 1, 1, 2, ct.c_void_p(G.data_ptr()), None) == L.E_INVALID
