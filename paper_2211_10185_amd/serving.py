"""Continuous-batching serving loop over the solver's C ABI.

Requests (one lattice problem each, k = 1 state) arrive over time.  The loop
keeps every admitted solve resident on the GPU and advances all of them
together one chunk (K imaginary-time steps) at a time with
``qfdtd_batch_evolve``; after each chunk it reads every solve's FP64 ground
energy with ``qfdtd_batch_energies`` and retires the solves whose energy moved
by less than ``tol`` since the previous chunk.  Requests that arrived in the
meantime are admitted at the next chunk boundary while device memory (by the
library's own footprint estimate) and slots allow, so their work overlaps with
the solves already running.

A request whose solve fails (a non-finite value or a collapsed norm, reported by
the library as QFDTD_E_NUMERIC) retires alone with status "failed" while the
others continue; a request for which ``should_cancel(rid)`` turns true retires at
the next chunk boundary with status "cancelled".
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import _lib as L
from . import solver as S


@dataclasses.dataclass
class Result:
    rid: int
    N: int
    kinetic: int
    energy: complex
    steps: int
    converged: bool
    t_arrival: float
    t_admit: float
    t_done: float
    psi: Optional[np.ndarray] = None
    status: str = "ok"          # "ok", "failed" or "cancelled"
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclasses.dataclass
class _Active:
    req: object
    solver: S.Solver
    footprint: int
    t_admit: float
    prev: Optional[complex] = None
    steps: int = 0


def serve(requests: Sequence, precision: int = S.C64, budget_bytes: Optional[int] = None,
          max_slots: int = 64, tol: float = 1e-8, max_steps: int = 50000, chunk: Optional[int] = None,
          keep_psi: bool = False, realtime: bool = True,
          clock: Callable[[], float] = time.perf_counter,
          should_cancel: Optional[Callable[[int], bool]] = None, init: str = "host",
          progress: Optional[Callable[[dict], None]] = None) -> dict:
    """Serve ``requests`` (objects with .rid, .arrival (s), .problem); return results and stats.

    ``realtime``: admit a request only once the wall clock has passed its arrival
    time; otherwise every request counts as arrived at t = 0 (a closed backlog).
    ``init``: "host" starts each solve from the problem's seeded host noise
    (``Problem.init_states``, uploaded); "device" from the library's seeded device noise
    (``qfdtd_set_state_noise`` with the problem's seed), with no host array.
    ``progress``: called after every chunk with the counts of finished, active and pending
    requests and the elapsed time.
    """
    import torch
    if budget_bytes is None:
        free, _total = torch.cuda.mem_get_info()
        budget_bytes = int(0.8 * free)
    pending = sorted(requests, key=lambda r: r.arrival)
    active: List[_Active] = []
    done: List[Result] = []
    used = 0
    peak_used = 0
    peak_active = 0
    chunks = 0
    # host time per part of the loop: admission (context creation and state upload), launching a
    # chunk, waiting for and reading the energies, retiring
    tpart = {"admit": 0.0, "launch": 0.0, "energies": 0.0, "retire": 0.0}
    t0 = clock()

    def now():
        return clock() - t0

    while pending or active:
        t = now()
        # admission: arrived requests, in arrival order, while slots and memory allow
        while pending and (not realtime or pending[0].arrival <= t) and len(active) < max_slots:
            p = pending[0].problem
            fp = S.footprint(p.N, p.kinetic, precision, p.k)
            if used + fp > budget_bytes and active:
                break
            req = pending.pop(0)
            ta = clock()
            sv = S.Solver.from_problem(p, precision=precision)
            _init(sv, p, init)
            active.append(_Active(req, sv, fp, now()))
            tpart["admit"] += clock() - ta
            used += fp
        peak_used = max(peak_used, used)
        peak_active = max(peak_active, len(active))
        if not active:
            # idle until the next arrival
            wait = pending[0].arrival - now()
            if wait > 0:
                time.sleep(min(wait, 0.01))
            continue
        if should_cancel is not None:
            keep = []
            for a in active:
                if should_cancel(a.req.rid):
                    done.append(_retire(a, None, False, realtime, now(), "cancelled", ""))
                    used -= a.footprint
                else:
                    keep.append(a)
            active = keep
            if not active:
                continue
        K = chunk or active[0].req.problem.measure_every
        dts = [a.req.problem.dt for a in active]
        tl = clock()
        try:
            S.batch_evolve([a.solver for a in active], K, dts)
            tpart["launch"] += clock() - tl
        except L.QfdtdError:
            # a member failed in an earlier chunk: batch_evolve checks every member before it
            # launches anything, so no solve advanced; retire the failed one(s) and go on
            keep = []
            for a in active:
                try:
                    a.solver.energies()
                    keep.append(a)
                except L.QfdtdError as err:
                    done.append(_retire(a, None, False, realtime, now(), "failed", str(err)))
                    used -= a.footprint
            if len(keep) == len(active):
                raise
            active = keep
            continue
        te = clock()
        try:
            E = list(S.batch_energies([a.solver for a in active])[:, 0])
            tpart["energies"] += clock() - te
        except L.QfdtdError:
            # every member advanced K steps; read them one by one (the same FP64 reductions, so
            # the same bits) and mark the failed one(s)
            E = []
            for a in active:
                try:
                    E.append(complex(a.solver.energies()[0]))
                except L.QfdtdError as err:
                    E.append(err)
        chunks += 1
        keep = []
        tr = clock()
        for a, e in zip(active, E):
            a.steps += K
            if isinstance(e, L.QfdtdError):
                done.append(_retire(a, None, False, realtime, now(), "failed", str(e)))
                used -= a.footprint
                continue
            conv = a.prev is not None and abs(e - a.prev) < tol
            if conv or a.steps >= max_steps:
                psi = a.solver.states(1)[1][0] if keep_psi else None
                done.append(Result(a.req.rid, a.req.problem.N, a.req.problem.kinetic, complex(e), a.steps, conv,
                                   a.req.arrival if realtime else 0.0, a.t_admit, now(), psi))
                a.solver.close()
                used -= a.footprint
            else:
                a.prev = complex(e)
                keep.append(a)
        active = keep
        tpart["retire"] += clock() - tr
        if progress is not None:
            progress({"done": len(done), "active": len(active), "pending": len(pending), "t": now()})
    makespan = now()
    ok = [r for r in done if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    svc = np.array([r.t_done - r.t_admit for r in ok]) if ok else np.zeros(1)
    return {"results": sorted(done, key=lambda r: r.rid), "makespan_s": makespan,
            "solves_per_s": len(ok) / makespan if makespan > 0 else 0.0,
            "failed": sum(r.status == "failed" for r in done),
            "cancelled": sum(r.status == "cancelled" for r in done),
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            # admission -> completion (time on the device, without queueing)
            "service_p50_s": float(np.percentile(svc, 50)), "service_p99_s": float(np.percentile(svc, 99)),
            "peak_active": peak_active, "peak_footprint_bytes": peak_used, "budget_bytes": budget_bytes,
            "chunks": chunks, "host_time_s": {k: round(v, 3) for k, v in tpart.items()}}


def _retire(a: _Active, e, conv: bool, realtime: bool, t: float, status: str, error: str) -> Result:
    a.solver.close()
    energy = complex(e) if e is not None else complex(np.nan, np.nan)
    return Result(a.req.rid, a.req.problem.N, a.req.problem.kinetic, energy, a.steps, conv,
                  a.req.arrival if realtime else 0.0, a.t_admit, t, None, status, error)


def _init(sv, p, init: str):
    if init == "device":
        sv.set_states_noise(p.seed)
    elif init == "host":
        sv.set_states(p.init_states())
    else:
        raise ValueError("init must be 'host' or 'device'")


def solve_alone(req, precision: int = S.C64, tol: float = 1e-8, max_steps: int = 50000,
                chunk: Optional[int] = None, keep_psi: bool = False, init: str = "host") -> Result:
    """The plain single-solve path: one request on its own, same stopping rule."""
    p = req.problem
    t0 = time.perf_counter()
    sv = S.Solver.from_problem(p, precision=precision)
    _init(sv, p, init)
    K = chunk or p.measure_every
    prev, steps, conv, e = None, 0, False, None
    while steps < max_steps:
        sv.evolve(K, p.dt)
        steps += K
        e = complex(sv.energies()[0])
        if prev is not None and abs(e - prev) < tol:
            conv = True
            break
        prev = e
    psi = sv.states(1)[1][0] if keep_psi else None
    sv.close()
    t1 = time.perf_counter()
    return Result(req.rid, p.N, p.kinetic, e, steps, conv, 0.0, 0.0, t1 - t0, psi)
