"""The split-x2 two-pass schedule (slab and pencil passes) against the oracle.

The x2 transform is split four-step style into a stride-16 part (slab pass, with the x3
transforms around the potential factor) and a consecutive-row part (pencil pass, with the x1
transforms around the kinetic factor), so one step is two passes over the state.  It computes
the same split-operator step as the other schedules (Sec. 2, eqs. HK1-HK3), in another
order of FP32 operations, so it is compared with the oracle, not bit for bit with them.
"""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from compare import energy_errors, wavefunction_errors

pytestmark = pytest.mark.gpu


def solver(p, **kw):
    from paper_2211_10185_amd.solver import Solver
    return Solver.from_problem(p, **kw)


@pytest.mark.parametrize("K,steps,variant", [(2, 4, 0), (1, 1, 0), (3, 5, 0), (2, 4, 1), (3, 5, 1),
                                             (2, 4, 2), (1, 1, 2), (3, 5, 2)])
def test_split_schedule_relativistic_cornell_256_matches_oracle(K, steps, variant):
    # complex V, parity sectors, chunks of one step and of odd length, both pencil tile widths
    p = S.config3()
    p.measure_every = K
    init = p.init_states()
    print("split schedule, 256^3 relativistic Cornell, K", K, "steps", steps, "variant", variant, flush=True)
    s = solver(p, split=True, split_variant=variant)
    assert s.schedule["split"]
    s.set_states(init)
    s.evolve(steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, steps=steps, init=init)
    print("energy err", np.max(energy_errors(E, ref["energies"])), flush=True)
    assert np.max(energy_errors(E, ref["energies"])) < 1e-5, (E, ref["energies"])
    assert np.max(wavefunction_errors(psi, ref["states"], ref["energies"])) < 1e-4


@pytest.mark.parametrize("kind,k", [(S.K_NR_SIN2, 3), (S.K_NR_P2, 1)])
def test_split_schedule_real_potential_256_matches_oracle(kind, k):
    a = 8.0 / 256
    p = S.Problem(N=256, a=a, m=1.0, kinetic=kind, vkind=S.V_HARMONIC, vparams=(1.0,), k=k,
                  precision=S.PREC_C64, dt=0.01, steps=3, measure_every=2, seed=77)
    init = p.init_states()
    print("split schedule, 256^3 harmonic, kind", kind, "k", k, flush=True)
    s = solver(p, split=True)
    s.set_states(init)
    s.evolve(p.steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, init=init)
    assert np.max(energy_errors(E, ref["energies"])) < 1e-5, (E, ref["energies"])
    assert np.max(wavefunction_errors(psi, ref["states"], ref["energies"])) < 1e-4


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_split_schedule_batch_and_graphs_give_the_bits_of_a_direct_solve(variant):
    from paper_2211_10185_amd.solver import batch_evolve
    p = S.config3()
    p.measure_every = 10
    q = S.Problem(N=64, a=0.125, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,), k=2,
                  precision=S.PREC_C64, dt=0.002, steps=0, measure_every=10, seed=3)
    print("split schedule: direct, graph replays, batch", flush=True)
    direct = solver(p, split=True, split_variant=variant, graphs=False)
    direct.set_states(p.init_states())
    direct.evolve(30, p.dt)
    Ed, pd = direct.states()
    direct.close()
    g = solver(p, split=True, split_variant=variant, graphs=True)
    g.set_states(p.init_states())
    for _ in range(3):                  # 10-step chunks: captured once, replayed twice
        g.evolve(10, p.dt)
        g.energies()
    Eg, pg = g.states()
    g.close()
    assert np.array_equal(Ed, Eg) and np.array_equal(pd, pg)
    a = solver(p, split=True, split_variant=variant)
    b = solver(q)
    a.set_states(p.init_states())
    b.set_states(q.init_states())
    batch_evolve([a, b], [30, 25], [p.dt, q.dt])
    Eb, pb = a.states()
    a.close()
    b.close()
    assert np.array_equal(Ed, Eb) and np.array_equal(pd, pb)


SPLIT_CASES = [  # N, kinetic, potential, split variant
    (96, S.K_REL, S.V_CORNELL, 0), (100, S.K_NR_P2, S.V_HARMONIC, 0), (108, S.K_NR_SIN2, S.V_CORNELL, 1),
    (120, S.K_REL, S.V_HARMONIC, 0), (128, S.K_REL, S.V_CORNELL, 0), (128, S.K_NR_SIN2, S.V_CORNELL, 2),
    (144, S.K_NR_SIN2, S.V_HARMONIC, 0), (150, S.K_REL, S.V_CORNELL, 0), (160, S.K_REL, S.V_CORNELL, 0),
    (160, S.K_NR_P2, S.V_CORNELL, 1), (162, S.K_NR_P2, S.V_HARMONIC, 1), (180, S.K_REL, S.V_CORNELL, 0),
    (192, S.K_NR_SIN2, S.V_CORNELL, 1), (216, S.K_REL, S.V_HARMONIC, 0), (240, S.K_REL, S.V_CORNELL, 0),
    (250, S.K_NR_SIN2, S.V_CORNELL, 0),
    # the two factors of x2 swapped
    (96, S.K_NR_P2, S.V_CORNELL, 3), (108, S.K_REL, S.V_HARMONIC, 3), (128, S.K_REL, S.V_CORNELL, 3),
    (144, S.K_NR_SIN2, S.V_CORNELL, 3), (150, S.K_REL, S.V_HARMONIC, 3), (160, S.K_REL, S.V_CORNELL, 3),
    (162, S.K_NR_SIN2, S.V_CORNELL, 3), (180, S.K_NR_P2, S.V_CORNELL, 3), (192, S.K_REL, S.V_CORNELL, 3),
    (216, S.K_NR_SIN2, S.V_HARMONIC, 3), (240, S.K_REL, S.V_CORNELL, 3), (250, S.K_REL, S.V_CORNELL, 3),
    (120, S.K_NR_SIN2, S.V_CORNELL, 3), (200, S.K_REL, S.V_CORNELL, 0), (200, S.K_NR_SIN2, S.V_HARMONIC, 3),
    (128, S.K_NR_P2, S.V_HARMONIC, 1)]


@pytest.mark.parametrize("N,kind,vkind,variant", SPLIT_CASES)
def test_split_schedule_every_split_size_matches_oracle(N, kind, vkind, variant):
    # x2 = N1 x N2 with radices 6, 8, 9, 10, 12, 15, 16, 18, 20 and 25 in the two parts; 2-column
    # pencil tiles where 4 does not divide N; 128-thread slab tiles up to N = 128.  The slab and
    # pencil kernels must be the ones that ran.
    a = 0.05
    vp = (0.4, 0.2, a / 2) if vkind == S.V_CORNELL else (1.0,)
    p = S.Problem(N=N, a=a, m=1.5, kinetic=kind, vkind=vkind, vparams=vp, k=2,
                  vgrid_seed=1031 if vkind == S.V_CORNELL else None, precision=S.PREC_C64,
                  dt=a / 8, steps=3, measure_every=2, seed=N)
    init = p.init_states()
    print("split schedule, N", N, "kind", kind, "vkind", vkind, "variant", variant, flush=True)
    s = solver(p, split=True, split_variant=variant)
    s.enable_kernel_timing(1)
    s.set_states(init)
    s.evolve(p.steps, p.dt)
    E, psi = s.states()
    n_slab = s.kernel_stats(5)[0]
    n_pencil = s.kernel_stats(6)[0]
    s.close()
    assert n_slab > 0 and n_pencil > 0, (n_slab, n_pencil)
    ref = O.solve(p, init=init)
    print("energy err", np.max(energy_errors(E, ref["energies"])), flush=True)
    assert np.max(energy_errors(E, ref["energies"])) < 1e-5, (E, ref["energies"])
    assert np.max(wavefunction_errors(psi, ref["states"], ref["energies"])) < 1e-4


@pytest.mark.parametrize("N,variant", [(160, 2), (256, 3)])
def test_split_variant_a_size_lacks_runs_the_plain_schedule(N, variant):
    # 160 has no 8-row variant and 256 = 16 x 16 no swapped one: the create call falls back to
    # the schedule the other flags select (row/column here), and no slab or pencil kernel runs
    a = 0.05
    p = S.Problem(N=N, a=a, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,), k=1,
                  precision=S.PREC_C64, dt=a / 8, steps=2, measure_every=2, seed=5)
    print("split variant fallback, N", N, "variant", variant, flush=True)
    s = solver(p, split=True, split_variant=variant, rowcol=True, groups=1)
    s.enable_kernel_timing(1)
    s.set_states(p.init_states())
    s.evolve(p.steps, p.dt)
    s.energies()
    counts = [s.kernel_stats(c)[0] for c in range(7)]
    s.close()
    assert counts[5] == 0 and counts[6] == 0 and counts[1] > 0, counts


@pytest.mark.parametrize("groups", [2, 3])
def test_split_schedule_state_groups_with_parity_sectors_match_oracle(groups):
    # config 3's structure at 128^3: complex V, sectors (P+, P+, P-_p3), the states split into
    # groups with their own pass chains on their own streams, chunks of 2 steps
    a = 0.05
    p = S.Problem(N=128, a=a, m=1.5, kinetic=S.K_REL, vkind=S.V_CORNELL, vparams=(0.4, 0.2, a / 2), k=3,
                  vgrid_seed=1031, sectors=(S.S_PLUS, S.S_PLUS, S.S_PK3), precision=S.PREC_C64,
                  dt=a / 8, steps=5, measure_every=2, seed=31)
    init = p.init_states()
    print("split schedule, 128^3, parity sectors, groups", groups, flush=True)
    s = solver(p, split=True, split_variant=0, groups=groups)
    assert s.schedule["groups"] == groups
    s.set_states(init)
    s.evolve(p.steps, p.dt)
    E, psi = s.states()
    s.close()
    ref = O.solve(p, init=init)
    print("energy err", np.max(energy_errors(E, ref["energies"])), flush=True)
    assert np.max(energy_errors(E, ref["energies"])) < 1e-5, (E, ref["energies"])
    assert np.max(wavefunction_errors(psi, ref["states"], ref["energies"])) < 1e-4


def test_batch_mixing_steady_and_chunk_edge_slab_passes_is_bitwise_alone():
    # two split members of one size with chunks of 4 and 6 steps: some slab launches hold one
    # member's chunk-end pass beside the other's steady pass (the two run as separate kernels);
    # a member of another split size rides along
    from paper_2211_10185_amd.solver import batch_evolve
    probs = [S.Problem(N=128, a=0.05, m=1.5, kinetic=S.K_REL, vkind=S.V_CORNELL, vparams=(0.3, 0.2, 0.025),
                       k=2, precision=S.PREC_C64, dt=0.05 / 8, steps=10, measure_every=4, seed=21),
             S.Problem(N=128, a=8.0 / 128, m=1.0, kinetic=S.K_NR_SIN2, vkind=S.V_HARMONIC, vparams=(1.0,),
                       k=1, precision=S.PREC_C64, dt=0.01, steps=13, measure_every=6, seed=22),
             S.Problem(N=160, a=8.0 / 160, m=1.0, kinetic=S.K_NR_P2, vkind=S.V_HARMONIC, vparams=(1.0,),
                       k=3, precision=S.PREC_C64, dt=0.01, steps=7, measure_every=5, seed=23)]
    print("batch of split members, chunks of 4, 6 and 5 steps", flush=True)
    alone = []
    for p in probs:
        s = solver(p, split=True)
        assert s.schedule["split"]
        s.set_states(p.init_states())
        s.evolve(p.steps, p.dt)
        alone.append(s.states())
        s.close()
    ss = [solver(p, split=True) for p in probs]
    for s, p in zip(ss, probs):
        s.set_states(p.init_states())
    batch_evolve(ss, [p.steps for p in probs], [p.dt for p in probs])
    for s, (Ea, psia) in zip(ss, alone):
        Eb, psib = s.states()
        s.close()
        assert np.array_equal(Ea, Eb)
        assert np.array_equal(psia, psib)
