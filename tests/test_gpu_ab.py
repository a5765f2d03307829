"""The A/B update with an FFT kinetic term (psi' = A psi - B dt H_K psi) on the GPU.

Element by element against the oracle's ``step_ab_fft`` on seeded inputs, for
the three FFT kinetic terms, both precisions and both pass schedules (plane +
column; row + three column passes), complex V and parity sectors; plus the
stability bound, bit-identical batching and graph replays.  Tolerances as for
the split step: complex128 to 1e-10 (energies) / 1e-9 (L2), complex64 to 1e-5 /
1e-4.
"""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from compare import energy_errors, phase_aligned_l2, wavefunction_errors

pytestmark = pytest.mark.gpu


def prob(kinetic, N, prec, vkind=S.V_HARMONIC, vparams=(1.0,), a=0.25, m=1.0, k=3, sectors=None,
         vgrid_seed=None, K=50, dt=None, seed=17):
    return S.Problem(N=N, a=a, m=m, kinetic=kinetic, vkind=vkind, vparams=vparams, k=k,
                     sectors=sectors, vgrid_seed=vgrid_seed, precision=prec,
                     dt=(a * a / 8 if dt is None else dt), steps=0, measure_every=K, seed=seed,
                     scheme=S.SCHEME_AB)


def cornell(N, prec, **kw):
    return prob(S.K_REL, N, prec, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5, dt=0.05 / 8, **kw)


CASES = [
    ("p2_ho32_c128", prob(S.K_NR_P2, 32, 1), 110, {}),
    ("p2_ho32_c64", prob(S.K_NR_P2, 32, 0), 110, {}),
    ("sin2_ho48_c64", prob(S.K_NR_SIN2, 48, 0, K=40), 110, {}),
    ("sin2_ho48_c64_rowcol", prob(S.K_NR_SIN2, 48, 0, K=40), 110, {"rowcol": True}),
    ("sin2_ho36_c128_rowcol", prob(S.K_NR_SIN2, 36, 1), 90, {"rowcol": True}),
    ("rel_cornell40_parity_complexV_c64", cornell(40, 0, sectors=(S.S_PLUS, S.S_PLUS, S.S_PK3), vgrid_seed=31), 100, {}),
    ("rel_cornell40_parity_complexV_c128", cornell(40, 1, sectors=(S.S_PLUS, S.S_PLUS, S.S_PK3), vgrid_seed=31), 100, {}),
    ("rel_cornell30_c64_rowcol", cornell(30, 0, k=2), 75, {"rowcol": True}),
]


@pytest.mark.parametrize("name,p,steps,kw", CASES, ids=[c[0] for c in CASES])
def test_ab_update_matches_oracle(name, p, steps, kw):
    from paper_2211_10185_amd.solver import Solver
    print("ab case", name, flush=True)
    init = p.init_states()
    s = Solver.from_problem(p, **kw)
    s.set_states(init)
    s.evolve(steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, steps=steps, init=init)
    if p.precision == 1:
        assert np.max(energy_errors(E, ref["energies"])) < 1e-10
        for i in range(p.k):
            assert phase_aligned_l2(psi[i], ref["states"][i]) < 1e-9
    else:
        assert np.max(energy_errors(E, ref["energies"])) < 1e-5
        assert np.max(wavefunction_errors(psi, ref["states"], ref["energies"])) < 1e-4


def test_ab_update_full_size_160_rowcol_sample():
    # N = 160 complex64 (the plane does not fit LDS): the row + column schedule, short run
    p = prob(S.K_NR_SIN2, 160, 0, a=0.1, k=1, K=6, dt=0.01 / 8)
    from paper_2211_10185_amd.solver import Solver
    init = p.init_states()
    s = Solver.from_problem(p)
    s.set_states(init)
    s.evolve(8, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, steps=8, init=init)
    assert np.max(energy_errors(E, ref["energies"])) < 1e-5
    assert phase_aligned_l2(psi[0], ref["states"][0]) < 1e-4


def test_ab_ho_converges_to_its_fixed_point():
    # 64^3 harmonic oscillator, H_K^(2), complex128: the converged energy is the A/B fixed point
    # (K + c V) psi = eps psi, c = 1 - dt eps / 2 (separable), within the convergence residual
    from paper_2211_10185_amd.solver import Solver
    N, a, m = 64, 0.25, 1.0
    p = prob(S.K_NR_SIN2, N, 1, k=1, dt=a * a / 8)
    x = O.coords(N, a)
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    D[0, -1] = D[-1, 0] = 1
    K1, V1 = -D / (2 * m * a * a), np.diag(0.5 * x * x)
    c = 1.0
    for _ in range(200):
        w_e, w_U = np.linalg.eigh(K1 + c * V1)
        c = 1 - p.dt * 3 * w_e[0] / 2
    w = w_U[:, 0]
    e_ref = 3 * (w @ (K1 + V1) @ w)
    s = Solver.from_problem(p)
    s.set_states(p.init_states())
    s.evolve(4000, p.dt)
    E = s.energies()
    s.close()
    assert abs(E[0].real - e_ref) < 1e-9, (E[0], e_ref)


@pytest.mark.parametrize("kind", [S.K_NR_P2, S.K_NR_SIN2, S.K_REL])
def test_ab_unstable_dt_is_rejected(kind):
    from paper_2211_10185_amd._lib import QfdtdError, E_UNSTABLE_DT
    from paper_2211_10185_amd.solver import Solver
    a, m = 0.2, 1.3
    p = prob(kind, 16, 0, a=a, m=m, k=1)
    bound = O.ab_dt_bound(kind, a, m)
    s = Solver.from_problem(p)
    s.set_states(p.init_states())
    with pytest.raises(QfdtdError) as ei:
        s.evolve(5, bound * 1.001)
    assert ei.value.status == E_UNSTABLE_DT
    s.evolve(5, bound * 0.999)
    assert np.all(np.isfinite(s.energies()))
    s.close()


def test_ab_and_split_members_batch_bitwise_equal_alone():
    from paper_2211_10185_amd.solver import Solver, batch_evolve
    probs = [prob(S.K_NR_SIN2, 48, 0, seed=1), cornell(40, 0, seed=2, K=7), prob(S.K_NR_P2, 64, 0, seed=3)]
    split = prob(S.K_NR_SIN2, 48, 0, seed=4)
    split.scheme = S.SCHEME_SPLIT
    probs.append(split)
    steps = [60, 33, 41, 50]
    # the same calls alone and in the batch (every call ends with an orthonormalisation)
    alone = []
    for p, n in zip(probs, steps):
        s = Solver.from_problem(p)
        s.set_states(p.init_states())
        s.evolve(n // 2, p.dt)
        s.evolve(n // 2, p.dt)
        if n % 2:
            s.evolve(n % 2, p.dt)
        alone.append(s.states())
        s.close()
    ss = [Solver.from_problem(p) for p in probs]
    for s, p in zip(ss, probs):
        s.set_states(p.init_states())
    for _ in range(2):                      # the second call replays the captured batch chunk
        batch_evolve(ss, [n // 2 for n in steps], [p.dt for p in probs])
    batch_evolve(ss, [n % 2 for n in steps], [p.dt for p in probs])
    for s, (Ea, pa) in zip(ss, alone):
        Eb, pb = s.states()
        assert np.array_equal(Ea, Eb)
        assert np.array_equal(pa, pb)
        s.close()


def test_ab_graph_replays_match_direct_launches():
    from paper_2211_10185_amd.solver import Solver
    p = prob(S.K_NR_P2, 40, 0, K=20)
    a = Solver.from_problem(p, graphs=True)
    b = Solver.from_problem(p, graphs=False)
    init = p.init_states()
    a.set_states(init)
    b.set_states(init)
    for rep in range(4):
        a.evolve(60, p.dt)
        b.evolve(60, p.dt)
        Ea, pa = a.states()
        Eb, pb = b.states()
        assert np.array_equal(Ea, Eb), rep
        assert np.array_equal(pa, pb), rep
    a.close()
    b.close()
