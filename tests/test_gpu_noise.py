"""Seeded device noise (qfdtd_set_state_noise) against the host implementation of the same
generator, and serving from it."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [1, 0])
def test_device_noise_equals_the_host_generator(prec):
    from paper_2211_10185_amd.solver import Solver
    N, k, seed = 24, 2, (5 << 32) + 11
    p = S.Problem(N=N, a=0.25, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,), k=k,
                  precision=prec, dt=0.01, steps=0, seed=seed)
    s = Solver.from_problem(p)
    s.set_states_noise(seed)
    got = np.stack([s.state_tensor(i).cpu().numpy().astype(np.complex128) for i in range(k)])
    s.close()
    want = S.philox_noise_states(N, k, seed)
    if prec == 0:
        want = want.astype(np.complex64).astype(np.complex128)
        assert np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3)) < 2.5e-7
    else:
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_serving_from_device_noise_matches_the_single_solve_path():
    from paper_2211_10185_amd.serving import serve, solve_alone
    reqs = S.config5(n_requests=4, rate=1000.0, seed=321)
    for q in reqs:
        q.problem.N = min(q.problem.N, 64)
        q.problem.a = 8.0 / q.problem.N
    out = serve(reqs, tol=1e-8, max_steps=3000, realtime=False, init="device")
    for r, q in zip(out["results"], reqs):
        alone = solve_alone(q, tol=1e-8, max_steps=3000, init="device")
        assert r.steps == alone.steps and r.energy == alone.energy
