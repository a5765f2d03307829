"""GPU path vs the FP64 oracle, element by element, on seeded inputs.

Sizes are small enough for the oracle to finish in seconds yet span several
tiles, ragged chunk ends (steps not a multiple of K) and both pass schedules
(plane + column for N <= 128 complex64 / N <= 96 complex128; row + 3 column
passes above).  Tolerances: complex128 paths to 1e-10; complex64 paths to the
stated budget, energies <= 1e-5 relative and wavefunctions <= 1e-4 in L2.
"""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from compare import energy_errors, phase_aligned_l2, wavefunction_errors

pytestmark = pytest.mark.gpu


def gpu_solver(p, precision=None, **kw):
    from paper_2211_10185_amd.solver import Solver
    return Solver.from_problem(p, precision=precision, **kw)


def run_both(p, steps, precision=None):
    prec = p.precision if precision is None else precision
    init = p.init_states()
    s = gpu_solver(p, precision=prec)
    s.set_states(init)
    s.evolve(steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, steps=steps, init=init)
    return E, psi, ref


def read_state(s, i):
    return s.state_tensor(i).cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("N,prec", [(32, 0), (48, 0), (80, 0), (96, 0), (128, 0), (160, 0), (250, 0), (256, 1),
                                    (36, 1), (64, 1), (96, 1), (100, 1), (128, 1)])
def test_transform_matches_oracle_dft(N, prec):
    from paper_2211_10185_amd.solver import Solver, NR_P2, V_HARMONIC
    print("transform N=%d prec=%d" % (N, prec), flush=True)
    s = Solver(N, 0.1, 1.0, NR_P2, V_HARMONIC, (1.0,), precision=prec, n_states=2)
    psi = S.initial_states(N, 2, 1000 + N)
    if prec == 0:
        psi = psi.astype(np.complex64).astype(np.complex128)
    s.set_states(psi)
    s.transform_state(1, -1)
    got = read_state(s, 1)
    ref = O.fft3(psi[1])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < (2e-6 if prec == 0 else 1e-13), err
    # state 0 untouched
    assert np.array_equal(read_state(s, 0), psi[0])
    s.transform_state(1, +1)
    back = read_state(s, 1)
    err2 = np.linalg.norm(back - psi[1]) / np.linalg.norm(psi[1])
    assert err2 < (4e-6 if prec == 0 else 1e-13), err2
    s.close()


def small(kinetic, N, prec, vkind=S.V_HARMONIC, vparams=(1.0,), a=0.25, m=1.0, k=3, sectors=None,
          vgrid_seed=None, K=50, dt=None, seed=7):
    return S.Problem(N=N, a=a, m=m, kinetic=kinetic, vkind=vkind, vparams=vparams, k=k,
                     sectors=sectors, vgrid_seed=vgrid_seed, precision=prec,
                     dt=(a * a / 8 if dt is None else dt), steps=0, measure_every=K, seed=seed)


CASES = [
    ("p2_ho32_c128", small(S.K_NR_P2, 32, 1), 120),
    ("p2_ho32_c64", small(S.K_NR_P2, 32, 0), 120),
    ("sin2_ho48_c64", small(S.K_NR_SIN2, 48, 0), 120),
    ("rel_cornell40_parity_c64", small(S.K_REL, 40, 0, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5,
                                        sectors=(S.S_PLUS, S.S_PLUS, S.S_PK3), vgrid_seed=31,
                                        dt=0.05 / 8), 110),
    ("rel_cornell40_parity_c128", small(S.K_REL, 40, 1, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5,
                                         sectors=(S.S_PLUS, S.S_PLUS, S.S_PK3), vgrid_seed=31,
                                         dt=0.05 / 8), 110),
    ("fdtd_ho32_c64", small(S.K_FDTD, 32, 0), 120),
    ("fdtd_ho30_c128_parity", small(S.K_FDTD, 30, 1, sectors=(S.S_PLUS, S.S_PK1, S.S_PK1)), 75),
    ("spline_p2_54_c64_k1", S.Problem(N=54, a=8 / 54, m=1.0, kinetic=S.K_NR_P2, vkind=S.V_RADIAL_SPLINE,
                                      knots=S.spline_knots(8.0, 5), k=1, precision=0, dt=0.01,
                                      steps=0, measure_every=50, seed=8), 130),
    ("sin2_ho144_4pass_c64", small(S.K_NR_SIN2, 144, 0, k=2, K=5), 12),
    ("rel_100_4pass_c128", small(S.K_REL, 100, 1, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5, k=2,
                                 K=4, dt=0.05 / 8), 10),
]


@pytest.mark.parametrize("name,p,steps", CASES, ids=[c[0] for c in CASES])
def test_small_solve_matches_oracle(name, p, steps):
    print("case", name, flush=True)
    E, psi, ref = run_both(p, steps)
    Er, psir = ref["energies"], ref["states"]
    if p.precision == 1:
        assert np.max(energy_errors(E, Er)) < 1e-10, (E, Er)
        for i in range(p.k):
            assert phase_aligned_l2(psi[i], psir[i]) < 1e-9
            # no phase fixing on either side: the arrays agree element by element
            assert np.max(np.abs(psi[i] - psir[i])) < 1e-9 * np.max(np.abs(psir[i]))
    else:
        assert np.max(energy_errors(E, Er)) < 1e-5, (E, Er)
        werr = wavefunction_errors(psi, psir, Er)
        assert np.max(werr) < 1e-4, werr


def test_config1_full_run_matches_oracle():
    p = S.config1()
    E, psi, ref = run_both(p, p.steps)
    Er = ref["energies"]
    assert np.max(energy_errors(E, Er)) < 1e-10, (E, Er)
    assert np.max(wavefunction_errors(psi, ref["states"], Er)) < 1e-8
    np.testing.assert_allclose(np.sort(E.real), [1.5, 2.5, 2.5], atol=2e-5)


ROW_CASES = [
    # one row tile holds the rows of all three states (the remainder path of the site index)
    ("rowcol_p2_ho8_c64", small(S.K_NR_P2, 8, 0, a=0.5, K=7), 30),
    # row tiles of 85 rows straddle the 144-row states (one wrap of the site index)
    ("rowcol_sin2_ho12_c128", small(S.K_NR_SIN2, 12, 1, a=0.5, K=7), 30),
    # tiles of 64 rows over 400-row states, complex potential
    ("rowcol_rel_cornell20_cV_c64", small(S.K_REL, 20, 0, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5,
                                          vgrid_seed=33, K=7, dt=0.05 / 8), 30),
    # N^2 a multiple of the tile height: whole tiles per state, so consecutive blocks take the
    # same rows of successive states (complex potential, then a real one in complex128)
    ("rowcol_rel_cornell32_cV_c64", small(S.K_REL, 32, 0, S.V_CORNELL, (0.4, 0.2, 0.025), a=0.05, m=1.5,
                                          vgrid_seed=35, K=7, dt=0.05 / 8), 30),
    ("rowcol_p2_ho32_c128", small(S.K_NR_P2, 32, 1, K=7), 30),
]


@pytest.mark.parametrize("name,p,steps", ROW_CASES, ids=[c[0] for c in ROW_CASES])
def test_row_schedule_small_lattices_match_oracle(name, p, steps):
    # the row + three column pass schedule forced on lattices whose planes would fit: row tiles
    # that span several states or straddle a state boundary
    print("case", name, flush=True)
    init = p.init_states()
    s = gpu_solver(p, rowcol=True)
    assert s.schedule["rowcol"]
    s.set_states(init)
    s.evolve(steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, steps=steps, init=init)
    Er, psir = ref["energies"], ref["states"]
    tol_e, tol_w = (1e-10, 1e-9) if p.precision == 1 else (1e-5, 1e-4)
    assert np.max(energy_errors(E, Er)) < tol_e, (E, Er)
    assert np.max(wavefunction_errors(psi, psir, Er)) < tol_w
