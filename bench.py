"""Benchmark: lattice site-updates/s of the imaginary-time evolution on one MI355X.

Default workload (one bench step = one whole solve): the relativistic Cornell
problem on a 256^3 periodic lattice (H_K^(3) = sqrt(p^2 + m^2) - m, m = 1.5,
a = 0.05, V = -0.4/r_f + 0.2 r_f with r_f = max(r, a/2), plus a seeded
imaginary part U(0, 0.01) drawn once per reflection orbit), 3 states in the
parity sectors (P+, P+, P-_p3), dt = a/8, 10000 steps, orthonormalisation and
parity projection every 50 steps, complex64 states with FP64 reductions, to its
three lowest complex energies.  The seeded initial states are resident in HBM
before the timed region; each bench step copies them in on the device, evolves
and reads back the energies.

Prints one JSON line.  value = site-updates/s = 3 states x 256^3 sites x 10000
steps / (seconds per bench step).  Other workloads: --workload ho128 (the
harmonic oscillator at 128^3 with FDTD and H_K^(2)), ab128, coulomb, batch64,
serve, dft16.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
CLASS_NAMES = {0: "plane_pass", 1: "row_pass", 2: "column_pass", 3: "fdtd_stencil", 5: "slab_pass",
               6: "pencil_pass"}
KERNEL_SYMBOLS = {0: "k_plane", 1: "k_row", 2: "k_col", 3: "k_stencil", 5: "k_slab", 6: "k_pencil"}
PASS_CLASSES = (0, 1, 2, 3, 5, 6)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--imag-steps", type=int, default=None,
                    help="imaginary-time steps per solve (default: 10000 for rel256, 5000 otherwise)")
    ap.add_argument("--timing-every", type=int, default=8, help="time one launch in this many")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-io", action="store_true", help="skip the PCIe-inclusive solve after the timed region")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="rel256",
                    choices=["ho128", "ab128", "coulomb", "rel256", "batch64", "serve", "dft16"],
                    help="rel256 (default): 256^3 relativistic Cornell solve with parity sectors and complex V; "
                         "ho128: the 128^3 harmonic oscillator with FDTD and H_K^(2); ab128: the same problem with H_K^(2) "
                         "stepped by the A/B update; coulomb: the Coulomb validation workload at 128^3; "
                         "batch64: 64 uneven Cornell solves in one batch; "
                         "serve: Poisson-arrival serving trace; "
                         "dft16: a batched 16-point DFT stage on the vector ALUs vs FP32 MFMA")
    ap.add_argument("--split", choices=["auto", "on", "off"], default="auto",
                    help="FFT solves: the split-x2 two-pass schedule where it exists (auto: the tuned choice)")
    ap.add_argument("--split-variant", type=int, choices=[0, 1, 2], default=None,
                    help="split-x2 variant: 0 = 4 x3 columns per pencil tile, 1 = 2, 2 = x2 = 32 x 8 with 8 "
                         "(default: the tuned choice)")
    ap.add_argument("--requests", type=int, default=1000, help="serve: number of requests in the trace")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrival rate (1/s)")
    ap.add_argument("--batch-steps", type=int, default=5000, help="batch64: imaginary-time steps")
    ap.add_argument("--no-fp64-path", action="store_true",
                    help="serve: skip the FP64 single-solve run of the same trace (for profiling the batched path)")
    return ap.parse_args()


def bench_batch(args):
    """64 independent Cornell solves of uneven N advanced together (one launch per pass kind and size)."""
    import numpy as np
    import torch
    import synthetic as S
    from paper_2211_10185_amd.solver import Solver, batch_evolve, batch_energies
    members = S.config4(n=64)
    solvers = [Solver.from_problem(p) for p in members]
    inits = []
    for s, p in zip(solvers, members):
        s.set_states(p.init_states())
    torch.cuda.synchronize()
    dts = [p.dt for p in members]
    batch_evolve(solvers, 50, dts)           # warm-up chunk
    batch_energies(solvers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch_evolve(solvers, args.batch_steps, dts)
    E = batch_energies(solvers)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sites = sum(p.k * p.N ** 3 for p in members)
    # after the timed region: one more chunk with every launch timed alone (HIP events attached to
    # the launch); a batched launch is charged to its first member's context
    for s in solvers:
        s.enable_kernel_timing(1)
    batch_evolve(solvers, 50, dts)
    batch_energies(solvers)
    torch.cuda.synchronize()
    dom, roof = roofline_of(solvers)
    roof["timing"] = "HIP events attached to every launch of one 50-step chunk after the timed region"
    roof["traffic"] = traffic_from_profiles("traffic_batch64.json", CLASS_NAMES[dom])
    for s in solvers:
        s.close()
    # algorithmic bytes per site-update: psi in and out (16 B) and the real FP32 factor shared by
    # the 3 states of a member (4/3 B)
    bps = 16.0 + 4.0 / 3.0
    return {"metric": "lattice site-updates/s", "value": sites * args.batch_steps / el, "unit": "site-updates/s",
            "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * el, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 Cornell solves, N drawn from {48,64,80,96,128,160}, kinetic H_K^(1..3) mixed, "
                                   "3 states, %d steps, complex64 + FP64 reductions" % args.batch_steps,
                       "sites_total": sites, "sizes": sorted({p.N for p in members})},
            "solves_per_s": len(members) / el,
            "energy_min_max": [float(np.min(E.real[:, 0])), float(np.max(E.real[:, 0]))],
            "roofline": roof,
            "path_roofline": {"bytes_per_su": round(bps, 3),
                              "R_alg": round(sites * args.batch_steps / el * bps / (PEAK_HBM_GBS * 1e9), 4)}}


def roofline_of(solvers):
    """Dominant pass class by total time (launch-attached HIP events), its algorithmic GB/s."""
    stats = {}
    for cls in PASS_CLASSES:
        cnt, tot_ms, tot_b = 0, 0.0, 0.0
        for s in solvers:
            n, mean_ms, b = s.kernel_stats(cls)
            cnt += n
            tot_ms += n * mean_ms
            tot_b += n * b
        if cnt:
            stats[cls] = (cnt, tot_ms / cnt, tot_b / cnt, tot_ms)
    dom = max(stats, key=lambda c: stats[c][3])
    cnt, mean_ms, bytes_per_launch, _ = stats[dom]
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                 "kernel": KERNEL_SYMBOLS[dom], "mean_launch_ms": round(mean_ms, 5),
            "timing": "HIP events attached to sampled launches during the last timed step, launches "
                      "not overlapped across streams",
                 "algorithmic_bytes_per_launch": bytes_per_launch, "timed_launches": cnt,
                 "by_class": {CLASS_NAMES[c]: {"mean_ms": round(v[1], 5),
                                               "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1),
                                               "share": round(v[3] / sum(x[3] for x in stats.values()), 3)}
                              for c, v in stats.items()}}


def bench_problem(args, p, workload, extra=None):
    """Site-updates/s of one solve of ``p`` per bench step (states resident on the device before
    timing); per-solve latency; launch-timed roofline of the dominant pass class."""
    import numpy as np
    import torch
    from paper_2211_10185_amd.solver import Solver
    from paper_2211_10185_amd import _lib
    N, k = p.N, p.k
    init_dev = torch.from_numpy(p.init_states().astype(np.complex64)).to("cuda")
    kw = {} if args.split == "auto" else {"split": args.split == "on"}
    if args.split_variant is not None:
        kw["split_variant"] = args.split_variant
    s = Solver.from_problem(p, **kw)

    def solve():
        for i in range(k):
            s._c(_lib.lib.qfdtd_set_state_device(s.ctx, i, init_dev[i].data_ptr()))
        s.evolve(p.steps, p.dt)
        return s.energies()

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for st in range(args.steps):
        if st == args.steps - 1:
            s.enable_kernel_timing(args.timing_every)   # last step: each timed launch runs alone
        t1 = time.perf_counter()
        E = solve()                                     # energies() synchronises
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dom, roof = roofline_of([s])
    s.enable_kernel_timing(0)
    value = k * N ** 3 * p.steps * args.steps / el
    lat_ms = sorted(1e3 * x for x in lat)
    out = {"metric": "lattice site-updates/s", "value": value, "unit": "site-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": workload, "N": N, "states": k, "imag_steps": p.steps},
           "solves_per_s": args.steps / el,
           "solve_latency_ms": {"p50": lat_ms[len(lat_ms) // 2],
                                "p99": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))]},
           "energies": [[round(e.real, 9), round(e.imag, 9)] for e in E], "roofline": roof}
    out.update(extra or {})
    return out, s, dom


def bench_ab(args):
    """The 128^3 harmonic problem with H_K^(2) stepped by the A/B update psi' = A psi - B dt H_K psi."""
    import synthetic as S
    p = S.config2(S.K_NR_SIN2)
    p.scheme = S.SCHEME_AB
    p.steps = args.imag_steps or 5000
    out, s, _ = bench_problem(args, p, "harmonic oscillator 128^3, a=0.25, m=1, 3 states, dt=a^2/8, %d steps, "
                                       "FFT H_K^(2) with the A/B update, complex64 states, FP64 reductions" % p.steps)
    s.close()
    # algorithmic: psi in and out (16 B) and the real FP32 factor shared by the 3 states (4/3 B);
    # pass model: column pass 16 B/SU + combine pass (alt, psi in; psi, alt out; V) 32 + 4/3 B/SU
    bsu = 16 + 4 / 3
    out["path_roofline"] = {"bytes_per_su": round(bsu, 3), "pass_bytes_per_su": round(48 + 4 / 3, 3),
                            "R_alg": round(out["value"] * bsu / (PEAK_HBM_GBS * 1e9), 4)}
    return out


def bench_coulomb(args):
    """Coulomb validation workload: 128^3, a = 0.12 fm, m = 0.3 GeV, alpha = 1, H_K^(2), 1s/2s/2p_z
    in the sectors (P+, P+, P^-_{p3}), run to tau = 80 fm; energies against -m alpha^2/(2 n^2)."""
    import oracle as O
    import synthetic as S
    p = S.coulomb_problem(S.K_NR_SIN2, N=128, a=0.12, alpha=1.0)
    out, s, _ = bench_problem(args, p, "Coulomb 128^3, a=0.12 fm, m=0.3 GeV, alpha=1, H_K^(2), sectors P+,P+,P-_p3, "
                                       "%d steps (tau=80 fm), complex64 states, FP64 reductions" % p.steps)
    s.close()
    th = [O.hydrogen_level(n, p.m, 1.0) for n in (1, 2, 2)]
    out["hydrogen_rel_error"] = [round((e[0] - t) / abs(t), 5) for e, t in zip(out["energies"], th)]
    return out


def bench_dft16(args):
    """Batched 16-point DFT stage, FP32: the solver's radix-16 butterfly on the vector ALUs against a
    dense 16 x 16 complex product on MFMA (v_mfma_f32_16x16x4_f32), 2^20 vectors of 16 points.
    reps = 64 repetitions in registers time the arithmetic; reps = 1 one stage between HBM read
    and write.  Accuracy: forward DFT (reps = 1) against torch's FP64 FFT."""
    import torch
    from paper_2211_10185_amd import dft_stage as D
    nvec = 1 << 20
    g = torch.Generator(device="cuda").manual_seed(16)
    x = torch.complex(torch.randn(nvec, 16, device="cuda", generator=g),
                      torch.randn(nvec, 16, device="cuda", generator=g)).contiguous()
    out = torch.empty_like(x)
    ref = torch.fft.fft(x.to(torch.complex128), dim=1)
    res = {}
    for name in ("valu", "mfma"):
        y = D.run(x, 1, name)
        err = ((y.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()
        rec = {"rel_err_fwd": err}
        for reps in (1, 64):
            D.time_launch(x, out, reps, name, iters=2)          # warm-up
            ms = D.time_launch(x, out, reps, name, iters=args.steps * 10)
            rec["reps%d" % reps] = {"ms": round(ms, 4), "dft16_per_s": nvec * reps / (ms * 1e-3)}
        res[name] = rec
    r64 = {k: res[k]["reps64"]["dft16_per_s"] for k in res}
    mfma_tflops = r64["mfma"] * 2048 / 1e12       # 16 MFMA x 2048 flops per tile of 16 vectors
    valu_nominal = r64["valu"] * 320 / 1e12       # 5 n log2 n nominal flops of a 16-point FFT
    return {
        "metric": "16-point DFT stage throughput (FP32, data in registers)", "value": r64["valu"],
        "unit": "DFT16/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2^20 vectors x 16 complex64 points, stage repeated 64 times in registers "
                               "(forward / inverse alternately), VALU butterfly vs MFMA 16x16 product",
                   "nvec": nvec},
        "variants": res,
        "valu_over_mfma": round(r64["valu"] / r64["mfma"], 3),
        "roofline": {"mfma": {"bound": "mfma", "achieved": round(mfma_tflops, 2), "peak": 157.3,
                              "unit": "TFLOP/s", "frac": round(mfma_tflops / 157.3, 4)},
                     "valu": {"bound": "alu", "achieved_nominal": round(valu_nominal, 2), "peak": 157.3,
                              "unit": "TFLOP/s", "frac": round(valu_nominal / 157.3, 4),
                              "note": "nominal 320 flops per DFT16 (5 n log2 n); the butterfly executes "
                                      "156 VALU instructions per DFT16 and lane"}},
    }


def bench_rel256(args):
    """256^3 with H_K^(3) = sqrt(p^2 + m^2) - m, Cornell V (alpha 0.4, sigma 0.2, m 1.5, a 0.05,
    r floored at a/2) plus a seeded imaginary part, three states in the sectors (P+, P+, P^-_{p3}),
    complex64 states with FP64 reductions, parity projection and orthonormalisation every 50
    steps; one whole solve per bench step."""
    import torch
    import synthetic as S
    p = S.config3()
    p.steps = args.imag_steps or 10000
    out, s, dom = bench_problem(args, p, "relativistic Cornell 256^3, a=0.05, m=1.5, H_K^(3) (rest mass removed), "
                                         "V=-0.4/r+0.2r (r floored at a/2) + i U(0,0.01) per reflection orbit, "
                                         "3 states in sectors P+,P+,P-_p3, dt=a/8, %d steps, complex64 states, "
                                         "FP64 reductions" % p.steps)
    out["config"]["reductions"] = "f64"
    split_names = {0: "x2 = 16 x 16, 4-column pencil tiles", 1: "x2 = 16 x 16, 2-column pencil tiles",
                   2: "x2 = 32 x 8, 8-column pencil tiles", 3: "x2 factors swapped"}
    out["config"]["schedule"] = ("split-x2 (slab + pencil passes, %s)" % split_names[s.schedule["split_variant"]]
                                 if s.schedule["split"] else "row + three column passes")
    out["roofline"]["traffic"] = traffic_from_profiles("traffic_rel256.json", CLASS_NAMES[dom])
    # algorithmic bytes per site-update: psi in and out (8 + 8 B) and the complex FP32 potential
    # factor, which the 3 states share, read once per step (8/3 B)
    bsu = 16 + 8 / 3
    out["path_roofline"] = {"bytes_per_su": round(bsu, 3), "R_alg": round(out["value"] * bsu / (PEAK_HBM_GBS * 1e9), 4),
                            "copy_ceiling_GBps": copy_ceiling_gbs()}
    # R_bw of the step: the counter-measured bytes of the step's two passes over their launch times
    moved = {c: traffic_from_profiles("traffic_rel256.json", CLASS_NAMES[c]) for c in (5, 6)}
    bc = out["roofline"]["by_class"]
    if all(moved.values()) and all(CLASS_NAMES[c] in bc for c in moved):
        t_step = sum(bc[CLASS_NAMES[c]]["mean_ms"] for c in moved) * 1e-3
        out["path_roofline"]["step_traffic_bytes"] = sum(moved.values())
        out["path_roofline"]["R_bw_step"] = round(sum(moved.values()) / t_step / (PEAK_HBM_GBS * 1e9), 4)
    out["device"] = device_record()
    if not args.no_host_io:
        # outside the timed region: the same solve with the states handed over in host memory
        # (complex128 upload, complex128 readback of states and energies): the PCIe-inclusive rate
        init = p.init_states()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_states(init)
        s.evolve(p.steps, p.dt)
        s.states()
        t_host = time.perf_counter() - t0
        out["host_io"] = {"value": p.k * p.N ** 3 * p.steps / t_host, "unit": "site-updates/s",
                          "note": "states uploaded from and read back to host memory (complex128) around the solve"}
    s.close()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_split(p, args.cpu_seconds)
    return out


def bench_serve(args):
    """Poisson serving trace: continuous batching in complex64 vs the plain FP64 single-solve path."""
    import numpy as np
    import synthetic as S
    from paper_2211_10185_amd.serving import serve, solve_alone
    reqs = S.config5(n_requests=args.requests, rate=args.rate)
    warm = S.config5(n_requests=2, rate=args.rate, seed=999)
    serve(warm, max_steps=200, init="device")
    last = [0.0]

    def report(st):
        # a progress line on stderr every 10 s, so a long trace shows that it advances
        if st["t"] - last[0] >= 10.0:
            last[0] = st["t"]
            print("serve: %d done, %d active, %d pending after %.0f s" % (st["done"], st["active"], st["pending"],
                                                                         st["t"]), file=sys.stderr, flush=True)

    out32 = serve(reqs, precision=0, init="device", progress=report)
    if args.no_fp64_path:
        return {"metric": "solves/s", "value": out32["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
                "steps": 1, "warmup": 1, "ms_per_step": 1e3 * out32["makespan_s"], "higher_is_better": True,
                "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "Poisson serving trace, %d requests at %.0f/s (batched complex64 path "
                                       "only)" % (args.requests, args.rate)},
                "latency_p50_s": out32["latency_p50_s"], "latency_p99_s": out32["latency_p99_s"],
                "chunks": out32["chunks"], "host_time_s": out32["host_time_s"]}
    t0 = time.perf_counter()
    alone64 = []
    for j, q in enumerate(reqs):
        alone64.append(solve_alone(q, precision=1, init="device"))
        if (j + 1) % 50 == 0:
            print("FP64 single solves: %d of %d after %.0f s" % (j + 1, len(reqs), time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    el64 = time.perf_counter() - t0
    # FP64 single-solve path on the same trace, requests served back to back in arrival order
    clock, lat64 = 0.0, []
    for q, r in zip(reqs, alone64):
        start = max(clock, q.arrival)
        clock = start + r.t_done
        lat64.append(clock - q.arrival)
    e32 = np.array([r.energy for r in out32["results"]])
    e64 = np.array([r.energy for r in alone64])
    rel = np.abs(e32 - e64) / np.maximum(np.abs(e64), 1e-2)
    return {"metric": "solves/s", "value": out32["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": 1e3 * out32["makespan_s"], "higher_is_better": True, "scaling": "strong",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "Poisson serving trace, %d requests at %.0f/s, N in even 2^a3^b5^c [32,256], "
                                   "spline potentials, k=1, dt=0.01, stop at |dE0|<1e-8, initial states from the "
                                   "library's seeded device noise (both paths)" % (args.requests, args.rate)},
            "latency_p50_s": out32["latency_p50_s"], "latency_p99_s": out32["latency_p99_s"],
            "service_p50_s": out32["service_p50_s"], "service_p99_s": out32["service_p99_s"],
            "peak_active": out32["peak_active"], "chunks": out32["chunks"], "host_time_s": out32["host_time_s"],
            "fp64_single_solve": {"solves_per_s": len(reqs) / el64, "latency_p50_s": float(np.percentile(lat64, 50)),
                                  "latency_p99_s": float(np.percentile(lat64, 99))},
            "fp32_vs_fp64_energy_rel_err": {"max": float(rel.max()), "median": float(np.median(rel))},
            "converged": int(sum(r.converged for r in out32["results"]))}


KERNEL_SOURCES = ("common.h", "fft_core.h", "fft_passes.h", "fft_inst.hip", "aux_kernels.hip")


def source_hash():
    """Hash of the device-kernel sources (the host library is left out: its changes do not move
    the profiled traffic)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2211_10185_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(fname, cls_name):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(cls_name)
    return None if k is None else k.get("bytes_per_launch")


def copy_ceiling_gbs(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (read + write bytes / s).  The default 1 GiB buffer is larger
    than the 256 MB on-package cache, so this is the practical HBM ceiling; a copy of the size of
    one state set (48 MiB at 128^3) stays in that cache and sets the ceiling the 128^3 passes
    actually stream against."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / t / 1e9, 1)


def device_record():
    """Device name and the current shader and memory clock levels, read from the driver's sysfs
    files (no helper program is started, so the bench runs unchanged under a profiler)."""
    import glob
    import torch
    rec = {"name": torch.cuda.get_device_name(0), "clocks": None}
    clocks = []
    for kind in ("sclk", "mclk"):
        for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_%s" % kind))[:1]:
            try:
                cur = [ln.strip() for ln in open(path) if ln.strip().endswith("*")]
            except OSError:
                cur = []
            if cur:
                clocks.append("%s %s" % (kind, cur[0].rstrip("* ").strip()))
    if clocks:
        rec["clocks"] = clocks
    return rec


def cpu_baseline(p_fdtd, p_fft, seconds):
    """The oracle, untuned, on a bounded sample of the same workload."""
    import numpy as np
    import oracle as O
    t_budget = seconds / 2
    res = {}
    total_su, total_t = 0.0, 0.0
    for p in (p_fdtd, p_fft):
        V = O.problem_potential(p)
        init = p.init_states()
        sectors = [0] * p.k
        periodic = p.kinetic != O.K_FDTD
        st = O.prepare(init, sectors, periodic)
        T = O.kinetic_symbol(p.kinetic, p.N, p.a, p.m) if periodic else None
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < t_budget:
            if periodic:
                st = [O.step_split(s, T, V, p.dt) for s in st]
            else:
                st = [O.step_fdtd(s, V, p.dt, p.a, p.m) for s in st]
            n += 1
        dt_ = time.perf_counter() - t0
        total_su += n * p.k * p.N ** 3
        total_t += dt_
        res[p.label] = n
    return {"value": total_su / total_t, "unit": "site-updates/s", "cores": O.WORKERS, "kind": "oracle",
            "sample": "FP64 numpy/scipy oracle steps of the same 128^3 x 3-state problems "
                      "(%d FDTD steps on one thread, %d FFT steps with %d FFT threads, %.0f s wall); "
                      "orthonormalisation excluded" % (res[p_fdtd.label], res[p_fft.label], O.WORKERS, total_t)}


def cpu_baseline_split(p, seconds):
    """The oracle, untuned, on a bounded sample of the same solve: FP64 split steps of all k states
    for about ``seconds`` of wall time (the factors exp(-dt V/2), exp(-dt T) computed once, as the
    oracle's own evolution loop does)."""
    import oracle as O
    V = O.problem_potential(p)
    sectors = list(p.sectors) if p.sectors else [0] * p.k
    st = O.prepare(p.init_states(), sectors, True)
    T = O.kinetic_symbol(p.kinetic, p.N, p.a, p.m)
    fac = O.split_factors(T, V, p.dt)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        st = [O.step_split(x, T, V, p.dt, fac) for x in st]
        n += 1
    el = time.perf_counter() - t0
    return {"value": n * p.k * p.N ** 3 / el, "unit": "site-updates/s", "cores": O.WORKERS, "kind": "oracle",
            "sample": "FP64 numpy/scipy oracle: %d split steps of the same %d-state %d^3 problem (%d FFT threads, "
                      "%.0f s wall); orthonormalisation and setup excluded" % (n, p.k, p.N, O.WORKERS, el)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(one lattice or one batch of lattices per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synthetic as S
    from paper_2211_10185_amd.solver import Solver

    torch.cuda.set_device(0)
    if args.workload == "batch64":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "ab128":
        print(json.dumps(bench_ab(args)), flush=True)
        return
    if args.workload == "coulomb":
        print(json.dumps(bench_coulomb(args)), flush=True)
        return
    if args.workload == "rel256":
        print(json.dumps(bench_rel256(args)), flush=True)
        return
    if args.workload == "dft16":
        print(json.dumps(bench_dft16(args)), flush=True)
        return
    dev = torch.device("cuda:0")
    imag = args.imag_steps or 5000
    p_fdtd = S.config2(S.K_FDTD)
    p_fft = S.config2(S.K_NR_SIN2)
    for p in (p_fdtd, p_fft):
        p.steps = imag
    N, k = p_fft.N, p_fft.k
    init = p_fft.init_states()        # same seed for both forms
    init_dev = torch.from_numpy(init.astype(np.complex64)).to(dev)
    solvers = [Solver.from_problem(p) for p in (p_fdtd, p_fft)]
    torch.cuda.synchronize()

    lat = []

    def one_step():
        out = []
        for s, p in zip(solvers, (p_fdtd, p_fft)):
            t0 = time.perf_counter()
            for i in range(k):
                s._c(s_lib.qfdtd_set_state_device(s.ctx, i, init_dev[i].data_ptr()))
            s.evolve(p.steps, p.dt)
            E = s.energies()
            lat.append(time.perf_counter() - t0)
            out.append(E)
        return out

    from paper_2211_10185_amd import _lib
    s_lib = _lib.lib

    for _ in range(args.warmup):
        one_step()
    lat.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(args.steps):
        if st == args.steps - 1:
            # launch timing in the last step: its launches run without the two-stream
            # overlap, so each timed kernel is measured alone, as the profiler sees it
            for s in solvers:
                s.enable_kernel_timing(args.timing_every)
        energies = one_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_per_step = 1e3 * elapsed / args.steps
    su_per_step = 2 * k * N ** 3 * imag
    value = su_per_step / (elapsed / args.steps)

    # dominant kernel class by total time in the timed region
    stats = {}
    for cls in PASS_CLASSES:
        cnt, tot_ms, tot_b = 0, 0.0, 0.0
        for s in solvers:
            n, mean_ms, b = s.kernel_stats(cls)
            cnt += n
            tot_ms += n * mean_ms
            tot_b += n * b
        if cnt:
            stats[cls] = (cnt, tot_ms / cnt, tot_b / cnt, tot_ms)
    dom = max(stats, key=lambda c: stats[c][3])
    cnt, mean_ms, bytes_per_launch, _ = stats[dom]
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles("traffic_ho128.json", CLASS_NAMES[dom])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": KERNEL_SYMBOLS[dom], "mean_launch_ms": round(mean_ms, 5),
            "timing": "HIP events attached to every %d-th launch during the last timed step, launches "
                      "not overlapped across streams" % args.timing_every,
            "algorithmic_bytes_per_launch": bytes_per_launch, "timed_launches": cnt,
            "by_class": {CLASS_NAMES[c]: {"mean_ms": round(v[1], 5), "GB/s": round(v[2] / (v[1] * 1e-3) / 1e9, 1),
                                          "share": round(v[3] / sum(x[3] for x in stats.values()), 3)}
                         for c, v in stats.items()}}
    lat_ms = sorted(1e3 * x for x in lat)
    out = {
        "metric": "lattice site-updates/s", "value": value, "unit": "site-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "harmonic oscillator 128^3, a=0.25, m=1, 3 states, dt=a^2/8, %d steps, "
                               "FDTD H_K^(0) + FFT H_K^(2), complex64 states, FP64 reductions" % imag,
                   "N": N, "states": k, "imag_steps": imag, "solves_per_step": 2,
                   "reductions": "f64"},
        "solves_per_s": 2 * args.steps / elapsed,
        "solve_latency_ms": {"p50": lat_ms[len(lat_ms) // 2], "p99": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))]},
        "energies": {"fdtd": [round(e.real, 9) for e in energies[0]], "sin2": [round(e.real, 9) for e in energies[1]]},
        "roofline": roof,
        # whole path: algorithmic bytes (16 + 4/3 B per site-update: read + write a complex64 site,
        # read the real FP32 potential factor that the 3 states share once per step) at the
        # measured rate, against the peak and a measured copy
        "path_roofline": {"bytes_per_su": round(16 + 4 / 3, 3),
                          "R_alg": round(value * (16 + 4 / 3) / (PEAK_HBM_GBS * 1e9), 4),
                          "copy_ceiling_GBps": copy_ceiling_gbs(),
                          "copy_ceiling_cache_resident_GBps": copy_ceiling_gbs(48 << 20, reps=40)},
        "device": device_record(),
    }
    # outside the timed region: one solve of each form with the states handed over in host
    # memory (FP64 upload, FP64 readback of states and energies): the PCIe-inclusive rate
    if not args.no_host_io:
        for s in solvers:
            s.enable_kernel_timing(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, p in zip(solvers, (p_fdtd, p_fft)):
            s.set_states(init)
            s.evolve(p.steps, p.dt)
            s.states()
        t_host = time.perf_counter() - t0
        out["host_io"] = {"value": su_per_step / t_host, "unit": "site-updates/s",
                          "note": "states uploaded from and read back to host memory (complex128) around each solve"}
    for s in solvers:
        s.close()
    if not args.no_cpu_baseline:
        pf = S.config2(S.K_FDTD)
        pk = S.config2(S.K_NR_SIN2)
        out["cpu_baseline"] = cpu_baseline(pf, pk, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
