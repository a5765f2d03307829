"""Excited states from snapshots of one evolving state (the legacy extraction, Sec. 1).

One state evolves alone and is normalised every chunk of steps.  The normalised state after
each chunk stays on the device as a snapshot S_j at tau_j; the last one is the ground state
phi0.  The first excited state comes from orthogonal projection of the snapshots against phi0:
E1(tau_j) is the energy of the projected snapshot.  While the higher levels decay, E1(tau)
falls; once the excited part of a snapshot sinks into the rounding of the projection it is
noise.  The value is read at the stationary point (the detection of the stabilisation of
E_i(tau) that Sec. 4 lists as future work): the minimum of E1(tau_j) over the snapshots whose
projected norm r_j stays above a rounding floor.  The second excited state repeats this with
the snapshots projected against phi0 and the first excited state found.

Every projection, norm and energy runs on the device through the C ABI (qfdtd_gram_residuals
gives r_j from the FP64 Cholesky factor of the Gram matrix, qfdtd_states the projection and the
energy); the host only compares numbers to pick the stationary point.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import solver as S

# unit roundoff of the state precision
EPS = {S.C64: 2.0 ** -23, S.C128: 2.0 ** -52}
# The device orthonormalisation factors the FP64 Gram matrix (Cholesky); the projected norm of a
# snapshot nearly parallel to the fixed states comes out of G_jj - |G_ij|^2 with an absolute
# error of about 1e-16 in r^2, so r is resolved only well above 1e-8.  Snapshots with a smaller
# projected norm are not used (their projection would be rounding, and near 1e-12 the library
# reports a collapsed norm).
MIN_RESIDUAL = 1e-7


def _stationary(E: np.ndarray, r: np.ndarray, floor: float) -> Optional[int]:
    best = None
    for j in range(len(E)):
        if r[j] > floor and np.isfinite(E[j]) and (best is None or E[j] < E[best]):
            best = j
    return best


def extract(problem, steps: int, every: Optional[int] = None, precision: Optional[int] = None,
            floor: Optional[float] = None, n_excited: int = 2) -> dict:
    """Snapshot extraction for ``problem`` (a synthetic.Problem; state 0 of its seeded initial
    states is evolved).  Returns taus, the ground energy, and per excited state the curve
    E_i(tau_j), the projected norms r_j, the stationary index and value."""
    prec = problem.precision if precision is None else int(precision)
    every = int(every or problem.measure_every)
    floor = max(1e3 * EPS[prec] if floor is None else float(floor), MIN_RESIDUAL)
    sec = (problem.sectors[0],) if problem.sectors else None
    one = dataclasses.replace(problem, k=1, sectors=sec, measure_every=every)
    main = S.Solver.from_problem(one, precision=prec)
    main.set_states(one.init_states())
    snaps, taus = [], []
    done = 0
    while done < steps:
        n = min(every, steps - done)
        main.evolve(n, problem.dt)
        done += n
        snaps.append(main.state_tensor(0).clone())
        taus.append(done * problem.dt)
    E0 = complex(main.energies()[0])
    main.close()
    phi0 = snaps[-1]
    fixed = [phi0]
    out = {"taus": np.array(taus), "E0": E0, "floor": floor, "levels": []}
    for _ in range(n_excited):
        kf = len(fixed)
        h = S.Solver.from_problem(dataclasses.replace(problem, k=kf + 1, sectors=None), precision=prec)
        E = np.full(len(snaps), np.nan)
        r = np.zeros(len(snaps))
        for j, sj in enumerate(snaps):
            for i, f in enumerate(fixed):
                h.set_state_device(i, f)
            h.set_state_device(kf, sj)
            r[j] = h.residuals()[kf]
            if r[j] > floor:
                E[j] = h.energies()[kf].real
        j_st = _stationary(E, r, floor)
        level = {"E": E, "r": r, "index": j_st, "value": None if j_st is None else float(E[j_st])}
        out["levels"].append(level)
        if j_st is None:
            h.close()
            break
        # the projected snapshot at the stationary point joins the fixed states
        for i, f in enumerate(fixed):
            h.set_state_device(i, f)
        h.set_state_device(kf, snaps[j_st])
        h.energies()
        fixed.append(h.state_tensor(kf).clone())
        h.close()
    return out
