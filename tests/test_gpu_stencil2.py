"""Two fused H_K^(0) steps per stencil pass against single-step passes, bit for bit.

The fused pass applies the update of eq. (HK0) twice in one sweep with the operations of the
single-step pass in the same order, so every run below must give identical bits with and
without it (QFDTD_F_STENCIL_1STEP).  The cases cover:
- the 128^3 workload;
- lattices that are not multiples of the 64 x 16 x 8 tile, and one smaller than a tile;
- a complex potential;
- chunks of odd length, where a pass of one step ends the chunk;
- a batch of uneven lattices;
- the largest lattice, 512^3.
Agreement with the FP64 oracle follows from the FDTD parity tests, which run the fused path.
"""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


def prob(N, k=3, K=50, vgrid_seed=None, seed=11, a=0.25):
    return S.Problem(N=N, a=a, m=1.0, kinetic=S.K_FDTD, vkind=S.V_HARMONIC, vparams=(1.0,), k=k,
                     precision=0, dt=a * a / 8, steps=0, measure_every=K, seed=seed, vgrid_seed=vgrid_seed)


def run(p, steps, fused, trace=False):
    from paper_2211_10185_amd.solver import Solver
    s = Solver.from_problem(p, fused_stencil=fused, trace=trace)
    s.set_states(p.init_states())
    s.evolve(steps, p.dt)
    E, psi = s.states()
    tr = s.energy_trace() if trace else None
    s.close()
    return E, psi, tr


@pytest.mark.parametrize("N,k,K,steps,vseed", [
    (128, 3, 50, 100, None),     # the 128^3 workload: 25 fused passes per chunk
    (40, 2, 7, 23, None),        # ragged tiles; chunks of 7 end with a single step
    (130, 1, 50, 9, 4),          # N not a multiple of 64 or 16, complex potential, odd count
    (8, 3, 4, 10, None),         # lattice smaller than one tile
    (66, 2, 1, 3, 2),            # chunks of one step only: no fused pass at all
])
def test_fused_passes_give_the_bits_of_single_steps(N, k, K, steps, vseed):
    print("stencil2 N=%d k=%d K=%d steps=%d vgrid_seed=%s" % (N, k, K, steps, vseed), flush=True)
    p = prob(N, k=k, K=K, vgrid_seed=vseed)
    E1, psi1, tr1 = run(p, steps, fused=False, trace=True)
    E2, psi2, tr2 = run(p, steps, fused=True, trace=True)
    assert np.array_equal(E1, E2)
    assert np.array_equal(psi1, psi2)
    assert np.array_equal(tr1, tr2)
    assert np.all(np.isfinite(E2.real)) and np.max(np.abs(psi2)) > 0


def test_fused_passes_in_a_batch_of_uneven_lattices():
    from paper_2211_10185_amd.solver import Solver, batch_evolve
    probs = [prob(48, k=3, K=50, seed=1), prob(100, k=2, K=9, seed=2), prob(20, k=1, K=50, seed=3, a=0.5)]
    steps = [50, 31, 17]
    print("stencil2 batch N=%s steps=%s" % ([p.N for p in probs], steps), flush=True)
    alone = [run(p, n, fused=False)[:2] for p, n in zip(probs, steps)]
    ss = [Solver.from_problem(p) for p in probs]
    for s, p in zip(ss, probs):
        s.set_states(p.init_states())
    batch_evolve(ss, steps, [p.dt for p in probs])
    for s, (Ea, psia) in zip(ss, alone):
        Eb, psib = s.states()
        s.close()
        assert np.array_equal(Ea, Eb)
        assert np.array_equal(psia, psib)


def test_fused_pass_at_the_largest_lattice():
    # N = 512 (2^27 sites, the largest H_K^(0) lattice): two steps as one fused pass against two
    # single-step passes, the whole state compared on the device; the single step at this size
    # is checked against the per-site oracle in the system tests
    import torch
    from paper_2211_10185_amd.solver import Solver, FDTD, V_HARMONIC
    N, a, m = 512, 0.05, 1.0
    dt = m * a * a / 8
    print("stencil2 N=512 two steps", flush=True)
    psi0 = S.initial_states(N, 1, 512)
    out = []
    for fused in (True, False):
        s = Solver(N, a, m, FDTD, V_HARMONIC, (1.0,), precision=0, n_states=1, measure_every=2,
                   fused_stencil=fused)
        s.set_states(psi0)
        s.evolve(2, dt)
        E = s.energies()
        out.append((E, s.state_tensor(0).clone()))
        s.close()
        torch.cuda.synchronize()
    assert np.array_equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    assert bool(torch.isfinite(torch.view_as_real(out[0][1])).all())
