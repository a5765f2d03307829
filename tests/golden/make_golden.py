"""Write the stored oracle results of the long runs (tests/golden/*.json, *.npz).

The FP64 oracle needs hours for these, so it runs once, here, and the GPU tests
compare against what it stored.  This script calls only ``oracle`` (the method)
and ``synthetic`` (the seeded inputs); nothing it stores comes from the HIP path.

Sets (paper: Sec. 2 eqs. HK1-HK3 for the kinetic terms and the split step,
Sec. 1 for the orthogonal projection of excited states, Sec. 3 for the parity
projectors):

* ``cfg3``: the 256^3 relativistic Cornell solve with the complex perturbation and
  the sectors (P+, P+, P-_p3), 10000 steps; energies every 1000 steps, sampled
  wavefunctions after 1000 and 10000 steps.
* ``cfg4``: the first member of every lattice size of the batch of 64, 5000 steps;
  energies and sampled wavefunctions.
* ``cfg5``: a stratified subset of 16 requests of the 1000-request serving trace
  (every kinetic kind, sizes across [32, 256]), each run to |dE0| < 1e-8 between
  50-step chunks; the step count, energy and sampled wavefunction at the stop.

Wavefunctions are stored at a seeded sample of sites rather than whole (a 256^3
state is 268 MB).  Sites are drawn with replacement from the mixture density
q(x) = 1/(2 N^3) + (1/(2k)) sum_i |psi_i(x)|^2 of the oracle's final states, so
sum_x f(x) is estimated without bias by mean_j f(x_j)/q(x_j): with f = |psi_gpu -
psi_oracle|^2 (after phase alignment, or after the best unitary within a
degenerate level) that is the squared L2 distance of the whole lattice.

Usage (resumable with --ckpt; checkpoints are whole FP64 states):
    python tests/golden/make_golden.py cfg4 cfg5 cfg3 [--ckpt DIR] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402
import oracle as O     # noqa: E402

SAMPLE_SEED = 4242


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def sample_sites(states: np.ndarray, n: int, seed: int):
    """Seeded draw of n flat site indices from q = 1/(2 N^3) + mean_i |psi_i|^2 / 2."""
    k = states.shape[0]
    n3 = states[0].size
    dens = np.zeros(n3)
    for i in range(k):
        dens += np.abs(states[i].ravel()) ** 2
    dens /= dens.sum()
    q = 0.5 / n3 + 0.5 * dens
    rng = np.random.Generator(np.random.PCG64(seed))
    uni = rng.random(n) < 0.5
    sites = np.empty(n, dtype=np.int64)
    sites[uni] = rng.integers(0, n3, size=int(uni.sum()))
    cdf = np.cumsum(dens)
    u = rng.random(int((~uni).sum())) * cdf[-1]
    sites[~uni] = np.minimum(np.searchsorted(cdf, u, side="right"), n3 - 1)
    return sites, q[sites]


def sample_record(states, n, seed):
    sites, q = sample_sites(states, n, seed)
    vals = np.stack([s.ravel()[sites] for s in states])      # [k, n]
    return {"sites": sites, "q": q.astype(np.float64),
            "psi_re": vals.real.astype(np.float32), "psi_im": vals.imag.astype(np.float32)}


def cplx(E):
    return [[float(np.real(e)), float(np.imag(e))] for e in E]


def problem_meta(p):
    return {"label": p.label, "N": p.N, "a": p.a, "m": p.m, "kinetic": p.kinetic,
            "vkind": p.vkind, "vparams": list(p.vparams), "k": p.k,
            "sectors": list(p.sectors) if p.sectors else None, "dt": p.dt,
            "measure_every": p.measure_every, "seed": p.seed}


def run_fixed(p, marks, ckpt, pool, tag, sample_at):
    """Oracle evolution of problem p; at each step count in ``marks`` the energies, and at the
    counts in ``sample_at`` ({mark: (n, seed)}) a site sample of the states.  Returns
    {mark: (E, sample record or None)}.  Resumable through ``ckpt``."""
    sectors = list(p.sectors) if p.sectors else [O.S_NONE] * p.k
    periodic = p.kinetic != O.K_FDTD
    V = O.problem_potential(p)
    done = 0
    out = {}
    path = os.path.join(ckpt, tag + ".npz") if ckpt else None
    marks_path = os.path.join(ckpt, tag + "_marks.npz") if ckpt else None
    if path and os.path.exists(path):
        z = np.load(path)
        states = list(z["states"])
        done = int(z["done"])
        log(tag, "resumed at", done)
        if os.path.exists(marks_path):
            z = np.load(marks_path)
            for mk in marks:
                if "E%d" % mk in z:
                    rec = None
                    if mk in sample_at:
                        rec = {key: z["S%d_%s" % (mk, key)] for key in ("sites", "q", "psi_re", "psi_im")}
                    out[mk] = (z["E%d" % mk], rec)
    else:
        states = O.prepare(p.init_states(), sectors, periodic)
    while done < marks[-1]:
        nxt = min(m for m in marks if m > done)
        # whole chunks of K only, so the orthonormalisation points match a single run
        seg = min(nxt - done, 500)
        seg = max(p.measure_every, (seg // p.measure_every) * p.measure_every)
        seg = min(seg, nxt - done)
        t0 = time.time()
        states = O.evolve(states, p.kinetic, p.a, p.m, V, p.dt, seg, p.measure_every, sectors,
                          None, getattr(p, "scheme", O.SCHEME_SPLIT), map_fn=pool.map)
        done += seg
        log(tag, "step", done, "%.2f s/step" % ((time.time() - t0) / seg))
        if done in marks:
            E = O.energies(states, p.kinetic, p.a, p.m, V)
            log(tag, "E at", done, E)
            rec = None
            if done in sample_at:
                n, seed = sample_at[done]
                rec = sample_record(np.stack(states), n, seed)
            out[done] = (E, rec)
        if path:
            flat = {}
            for mk, (E, rec) in out.items():
                flat["E%d" % mk] = E
                if rec is not None:
                    for key, v in rec.items():
                        flat["S%d_%s" % (mk, key)] = v
            np.savez(marks_path + ".tmp.npz", **flat)
            os.replace(marks_path + ".tmp.npz", marks_path)
            np.savez(path + ".tmp.npz", states=np.stack(states), done=done)
            os.replace(path + ".tmp.npz", path)
    return out


def write(name, meta, arrays):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    np.savez_compressed(os.path.join(HERE, name + ".npz"), **arrays)
    log("wrote", name)


def cfg3(ckpt, pool):
    p = S.config3()
    marks = list(range(1000, p.steps + 1, 1000))
    sample_at = {mk: (2048, SAMPLE_SEED + mk) for mk in (1000, p.steps)}
    res = run_fixed(p, marks, ckpt, pool, "cfg3", sample_at)
    meta = {"what": "oracle.evolve/energies of the 256^3 relativistic Cornell solve (Sec. 2 eq. HK3; "
                    "Sec. 3 projectors P+, P-_p3; Sec. 1 orthogonal projection)",
            "problem": problem_meta(p), "vgrid_seed": p.vgrid_seed,
            "energies": {str(mk): cplx(res[mk][0]) for mk in marks}}
    arrays = {}
    for mk in sample_at:
        for key, v in res[mk][1].items():
            arrays["s%d_%s" % (mk, key)] = v
    meta["samples"] = [1000, p.steps]
    write("cfg3_cornell256_rel", meta, arrays)


def cfg4_pick():
    pick, seen = [], set()
    for j, p in enumerate(S.config4(n=64)):
        if p.N not in seen:
            seen.add(p.N)
            pick.append((j, p))
    return pick


def cfg4(ckpt, pool):
    meta = {"what": "oracle.evolve/energies of one member per lattice size of the batch of 64 Cornell "
                    "solves, 5000 steps (Sec. 2 eqs. HK1-HK3; Sec. 1 orthogonal projection)",
            "members": []}
    arrays = {}
    for j, p in cfg4_pick():
        res = run_fixed(p, [p.steps], ckpt, pool, "cfg4_%02d" % j, {p.steps: (1024, SAMPLE_SEED + j)})
        E, rec = res[p.steps]
        meta["members"].append({"index": j, "problem": problem_meta(p), "steps": p.steps,
                                "energies": cplx(E)})
        for key, v in rec.items():
            arrays["m%02d_%s" % (j, key)] = v
    write("cfg4_batch_members", meta, arrays)


def cfg5_pick(n_pick=16):
    """Stratified subset: per kinetic kind, requests at evenly spaced ranks of N."""
    reqs = S.config5(n_requests=1000)
    per_kind = {S.K_NR_P2: 6, S.K_NR_SIN2: 5, S.K_REL: 5}
    out = []
    for kind, cnt in per_kind.items():
        rs = sorted((r for r in reqs if r.problem.kinetic == kind), key=lambda r: (r.problem.N, r.rid))
        idx = np.round(np.linspace(0, len(rs) - 1, cnt)).astype(int)
        out += [rs[i] for i in idx]
    assert len(out) == n_pick
    return sorted(out, key=lambda r: r.rid)


def cfg5(ckpt, pool):
    meta = {"what": "oracle.solve_until_converged of a stratified 16-request subset of the 1000-request "
                    "serving trace (seed 105): |dE0| < 1e-8 between 50-step chunks (Sec. 2 eqs. HK1-HK3)",
            "tol": 1e-8, "requests": []}
    arrays = {}
    for r in cfg5_pick():
        p = r.problem
        t0 = time.time()
        res = O.solve_until_converged(p, tol=1e-8, max_steps=p.steps)
        log("cfg5 rid", r.rid, "N", p.N, "kind", p.kinetic, "steps", res["steps"],
            "E0", res["energies"][0], "%.0f s" % (time.time() - t0))
        meta["requests"].append({"rid": r.rid, "problem": problem_meta(p), "steps": int(res["steps"]),
                                 "energies": cplx(res["energies"])})
        rec = sample_record(res["states"], 1024, SAMPLE_SEED + 7 * r.rid)
        for key, v in rec.items():
            arrays["r%04d_%s" % (r.rid, key)] = v
    write("cfg5_serving_subset", meta, arrays)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sets", nargs="+", choices=["cfg3", "cfg4", "cfg5"])
    ap.add_argument("--ckpt", default=None, help="directory for resumable FP64 checkpoints")
    ap.add_argument("--threads", type=int, default=3, help="states stepped concurrently")
    args = ap.parse_args()
    if args.ckpt:
        os.makedirs(args.ckpt, exist_ok=True)
    with ThreadPoolExecutor(args.threads) as pool:
        for s in args.sets:
            {"cfg3": cfg3, "cfg4": cfg4, "cfg5": cfg5}[s](args.ckpt, pool)


if __name__ == "__main__":
    main()
