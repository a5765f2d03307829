"""Snapshot extraction of excited states (the legacy method) on the GPU.

The device E1(tau_j) curve and projected norms against the oracle's on the same seeded input
(complex128), the stationary values against the exact levels of a separable anisotropic
oscillator, and the single-precision failure of the method beside the block method, which
reaches the complex64 budget on the same problem.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

OMEGAS = (1.0, 1.3, 1.7)


def aniso(prec, N=16, a=0.5, m=1.0):
    return S.Problem(N=N, a=a, m=m, kinetic=S.K_NR_SIN2, vkind=S.V_GRID, k=1, dt=a * a / 8, steps=0,
                     seed=21, grid=S.anisotropic_ho_grid(N, a, OMEGAS), precision=prec, measure_every=50)


def exact_levels(N, a, m):
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    D[0, -1] = D[-1, 0] = 1
    x = O.coords(N, a)
    eps = [np.linalg.eigvalsh(-D / (2 * m * a * a) + np.diag(0.5 * w * w * x * x)) for w in OMEGAS]
    base = sum(e[0] for e in eps)
    ex = sorted([base + e[1] - e[0] for e in eps] + [base + e[2] - e[0] for e in eps])
    return base, ex[0], ex[1]


def test_snapshot_curve_matches_oracle_and_exact_levels_fp64():
    from paper_2211_10185_amd.snapshots import extract
    p = aniso(1)
    e0, e1, e2 = exact_levels(p.N, p.a, p.m)
    out = extract(p, 4000, 50)
    snaps, taus = O.snapshot_run(p, 4000, 50)
    E1o, r1o = O.snapshot_energies(p, snaps, [snaps[-1]])
    lv = out["levels"][0]
    np.testing.assert_allclose(out["taus"], taus, rtol=1e-14)
    # the snapshots the device uses (projected norm above its floor of 1e-7): energies agree with
    # the oracle's MGS projection to 1e-8, norms to the 1e-16 / r of the Gram-based residual
    sel = r1o > 1e-7
    assert sel.sum() >= 8
    assert np.max(np.abs(lv["E"][sel] - E1o.real[sel])) < 1e-8
    assert np.max(np.abs(lv["r"][sel] - r1o[sel])) < 5e-9
    assert abs(out["E0"].real - e0) < 1e-7
    # the stationary point lies where the projected norm reaches the floor: E1 to about 1e-4,
    # the second level (projected against two states) to about 1e-2
    print("fp64 snapshot E1 - e1 = %.3e at tau %.2f, E2 - e2 = %.3e" % (
        lv["value"] - e1, out["taus"][lv["index"]], out["levels"][1]["value"] - e2), flush=True)
    assert 0 < lv["value"] - e1 < 2e-4, (lv["value"], e1)
    v2 = out["levels"][1]["value"]
    assert 0 < v2 - e2 < 5e-2, (v2, e2)


def test_snapshot_fp32_failure_beside_the_block_method():
    from paper_2211_10185_amd.snapshots import extract
    from paper_2211_10185_amd.solver import Solver
    p = aniso(0)
    e0, e1, e2 = exact_levels(p.N, p.a, p.m)
    out = extract(p, 4000, 50)
    v1 = out["levels"][0]["value"]
    print("fp32 snapshot E1 - e1 = %.3e at tau %.2f" % (v1 - e1, out["taus"][out["levels"][0]["index"]]), flush=True)
    # the excited part of late complex64 snapshots is rounding: the method stops far short of
    # the complex64 budget
    assert 1e-3 < v1 - e1 < 2e-2, v1 - e1
    # three states evolved together and orthonormalised every 50 steps: within the budget
    q = dataclasses.replace(p, k=3)
    s = Solver.from_problem(q)
    s.set_states(q.init_states())
    s.evolve(4000, q.dt)
    E = s.energies().real
    s.close()
    for got, ref in zip(E, (e0, e1, e2)):
        assert abs(got - ref) < 1e-5 * abs(ref), (got, ref)


def test_gram_residuals_are_the_projected_norms():
    # psi_0 = 2 u0, psi_1 = 0.5 u0 + 0.3 u1, psi_2 = u0 - u1 + 1e-5 u2 with orthonormal u: the norms
    # after projection against the earlier states are 2, 0.3 and 1e-5
    from paper_2211_10185_amd.solver import Solver
    N = 16
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((N ** 3, 3)) + 1j * rng.standard_normal((N ** 3, 3)))
    u = U.T.reshape(3, N, N, N)
    states = np.stack([2 * u[0], 0.5 * u[0] + 0.3 * u[1], u[0] - u[1] + 1e-5 * u[2]])
    p = S.Problem(N=N, a=0.5, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,), k=3,
                  precision=1, dt=0.01, steps=0, seed=1)
    s = Solver.from_problem(p)
    s.set_states(states)
    r = s.residuals()
    G = s.gram()
    s.close()
    np.testing.assert_allclose(r[:2], [2.0, 0.3], rtol=1e-12)
    assert abs(r[2] - 1e-5) < 1e-10, r
    # the same from the Schur complement of the Gram matrix on the host
    r2 = G[2, 2].real - np.real(np.conj(G[:2, 2]) @ np.linalg.solve(G[:2, :2], G[:2, 2]))
    assert abs(np.sqrt(r2) - r[2]) < 1e-10
