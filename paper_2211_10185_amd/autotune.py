"""Pass-schedule autotuner for the FFT kinetic terms.

For a lattice size N, a state precision and a state count, the solver can run a
step as
  * the plane schedule (x2-x3 plane pass + x1 column pass: 2 passes per step),
    available where an N^2 plane fits in LDS, or
  * the row/column schedule (x3 row pass + three column passes: 4 passes), or
  * the split-x2 schedule (slab pass + pencil pass: 2 passes), for the sizes
    that have split-x2 kernels, with pencil tiles of 4 or 2 x3 columns, and at
    N = 128 and 256 also with 8-row tiles of 8 columns, and with the two factors
    of x2 swapped (a radix-plan choice),
and, with k >= 2 states, either carry all states through one stream or split
them into two (or, with k >= 3, three) groups pipelined on their own streams.  ``tune`` times every candidate
on the device with the solver's own kernels and records the fastest in a JSON
cache; ``schedule_for`` is what ``Solver`` consults at creation.

Cache: ``$QFDTD_TUNING`` if set, else ``tuning.json`` next to this file.
Entry key: "N/precision/states" with states clipped to {1, 2+}.  An entry with a "pinned" note
was chosen from another measurement (the note says which) and ``tune`` leaves it as it is.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
PLANE_LIMIT = {0: 128, 1: 96}      # largest N whose plane fits LDS (complex64 / complex128)
# sizes with split-x2 (slab and pencil) kernels
SPLIT_SIZES = {0: (96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192, 200, 216, 240, 250, 256), 1: ()}
SPLIT_WIDE_SIZES = {0: (128, 256), 1: ()}    # ... and with the 8-row, 8-column variant
SPLIT_SWAPPED_SIZES = {0: (96, 108, 120, 128, 144, 150, 160, 162, 180, 192, 200, 216, 240, 250), 1: ()}
_cache: Optional[Dict[str, dict]] = None


def cache_path() -> str:
    return os.environ.get("QFDTD_TUNING", os.path.join(HERE, "tuning.json"))


def _load() -> Dict[str, dict]:
    global _cache
    if _cache is None:
        try:
            with open(cache_path()) as f:
                _cache = json.load(f).get("entries", {})
        except (OSError, ValueError):
            _cache = {}
    return _cache


def key(N: int, precision: int, k: int) -> str:
    return "%d/%d/%d" % (N, precision, 1 if k <= 1 else 2)


def default_schedule(N: int, kinetic: int, precision: int, k: int) -> dict:
    # without a measurement: two streams pay off only once a group's passes fill the GPU
    single = k < 2 or N < 96
    return {"rowcol": False, "single_stream": single, "groups": 1 if single else 2, "split": False}


def schedule_for(N: int, kinetic: int, precision: int, k: int) -> dict:
    """Tuned schedule if the cache has one for (N, precision, k), else the default."""
    if kinetic == 0:
        return {"rowcol": False, "single_stream": True, "groups": 1, "split": False}
    e = _load().get(key(N, precision, k))
    if e is None:
        return default_schedule(N, kinetic, precision, k)
    single = bool(e["single_stream"])
    return {"rowcol": bool(e["rowcol"]), "single_stream": single,
            "groups": 1 if single else int(e.get("groups", 2)), "split": bool(e.get("split", False)),
            "split_variant": int(e.get("split_variant", 0))}


def candidates(N: int, precision: int, k: int):
    out = []
    plane_ok = N <= PLANE_LIMIT[precision]
    for rowcol in ([False, True] if plane_ok else [True]):
        groups = [1] if rowcol or k < 2 else ([1, 2, 3] if k >= 3 else [1, 2])
        for g in groups:
            out.append({"rowcol": rowcol, "single_stream": g == 1, "groups": g, "split": False})
    if N in SPLIT_SIZES[precision]:
        # variant 1 (2-column tiles) differs from variant 0 only where 4 divides N
        variants = ([0] + ([1] if N % 4 == 0 else []) + ([2] if N in SPLIT_WIDE_SIZES[precision] else [])
                    + ([3] if N in SPLIT_SWAPPED_SIZES[precision] else []))
        groups = [1, 2, 3] if k >= 3 else ([1, 2] if k >= 2 else [1])
        for v in variants:
            for g in groups:
                out.append({"rowcol": False, "single_stream": g == 1, "groups": g, "split": True,
                            "split_variant": v})
    return out


def candidate_name(c: dict, N: int = 256) -> str:
    if c.get("split"):
        v = c.get("split_variant", 0)
        cols = 4 if N % 4 == 0 else 2
        name = {0: "split/%dcol" % cols, 1: "split/2col", 2: "split8row/8col", 3: "split-swapped"}[v]
        return name + ("" if c.get("groups", 1) == 1 else "/%dstreams" % c["groups"])
    return ("rowcol" if c["rowcol"] else "plane") + ("/1stream" if c["groups"] == 1 else "/%dstreams" % c["groups"])


def time_schedule(N: int, precision: int, k: int, sched: dict, steps: int = 400, kinetic: int = 2,
                  reps: int = 2) -> float:
    """Microseconds per imaginary-time step of a harmonic problem under `sched` (the best of
    `reps` timed runs of `steps` steps, after a warm-up chunk that also captures the graph)."""
    import torch
    import synthetic as S
    from .solver import Solver
    a = 8.0 / N
    s = Solver(N, a, 1.0, kinetic, S.V_HARMONIC, (1.0,), precision=precision, n_states=k,
               rowcol=sched["rowcol"], groups=sched.get("groups", 1 if sched["single_stream"] else 2),
               split=sched.get("split", False), split_variant=sched.get("split_variant", 0))
    s.set_states(S.initial_states(N, k, 7))
    dt = a * a / 8
    s.evolve(50, dt)
    s.energies()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        s.evolve(steps, dt)
        s.energies()
        torch.cuda.synchronize()
        best = min(best, 1e6 * (time.perf_counter() - t0) / steps)
    s.close()
    return best


def tune(sizes: Iterable[int], precisions: Iterable[int] = (0,), states: Iterable[int] = (1, 3),
         steps: int = 400, path: Optional[str] = None, verbose: bool = True) -> Dict[str, dict]:
    """Time every candidate schedule and write the winners to the cache."""
    global _cache
    path = path or cache_path()
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        doc = {"entries": {}}
    entries = doc.setdefault("entries", {})
    for N in sizes:
        for prec in precisions:
            for k in states:
                if entries.get(key(N, prec, k), {}).get("pinned"):
                    # a choice made from a measurement other than this timing (the entry says which)
                    if verbose:
                        print("tune N=%d prec=%d k=%d: pinned, kept" % (N, prec, k), flush=True)
                    continue
                times, cands = {}, {}
                for c in candidates(N, prec, k):
                    name = candidate_name(c, N)
                    cands[name] = c
                    times[name] = time_schedule(N, prec, k, c, steps)
                best = min(times, key=times.get)
                c = cands[best]
                entries[key(N, prec, k)] = {"rowcol": c["rowcol"], "single_stream": c["groups"] == 1,
                                            "groups": c["groups"], "split": c["split"],
                                            "split_variant": c.get("split_variant", 0),
                                            "us_per_step": {n: round(v, 2) for n, v in times.items()}}
                if verbose:
                    print("tune N=%d prec=%d k=%d -> %s %s" % (N, prec, k, best, entries[key(N, prec, k)]["us_per_step"]),
                          flush=True)
    doc["device"] = _device_name()
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    _cache = None
    return entries


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


if __name__ == "__main__":
    import argparse
    import synthetic as S
    ap = argparse.ArgumentParser(description="time the candidate schedules of every FFT lattice size")
    ap.add_argument("out", nargs="?", default=None, help="cache file to write (default: tuning.json here)")
    ap.add_argument("--steps", type=int, default=400, help="timed imaginary-time steps per run")
    ap.add_argument("--sizes", type=int, nargs="*", default=None, help="lattice sizes (default: 32..256)")
    ap.add_argument("--precisions", type=int, nargs="*", default=[0, 1], help="0: complex64, 1: complex128")
    a = ap.parse_args()
    sizes = a.sizes or [n for n in S.smooth_even_sizes(32, 256)]
    tune(sizes, precisions=a.precisions, states=(1, 3), steps=a.steps, path=a.out)
