"""Seeded synthetic inputs for the imaginary-time Schroedinger workloads.

This module is the only code shared by the FP64 oracle and the GPU path.  It
draws random numbers and lays out problem descriptions; it holds none of the
method's arithmetic (no potentials evaluated, no transforms, no stencils, no
reductions).  Every array it returns is an *input*: initial wavefunctions,
per-site random perturbations, spline knots, batch members, arrival traces.

Random streams: numpy ``Generator(PCG64(seed))``.  For a k-state initial
condition the draws are, for each state in order, the real part then the
imaginary part, each ``standard_normal(N**3)`` in C order (x1 slowest, x3
fastest).

Lattice convention shared by both sides (the paper writes Psi(r) for
Psi[(A x1, A x2, A x3)], Sec. 2): site index i_l in [0, N), coordinate
x_l = (i_l - N/2) * a, so the origin sits on site N/2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Kinetic-term identifiers, H_K^(0..3) of Sec. 2 (eqs. HK0..HK3).
K_FDTD = 0      # 7-point finite-difference Laplacian, Dirichlet walls
K_NR_P2 = 1     # FFT, sum_l k_l^2 / (2 A^2 M)
K_NR_SIN2 = 2   # FFT, sum_l 4 sin^2(k_l/2) / (2 A^2 M)
K_REL = 3       # FFT, sqrt(4 sum sin^2(k_l/2)/A^2 + M^2) (evolved with -M)

# Potential identifiers.
V_GRID = 0
V_HARMONIC = 1
V_CORNELL = 2
V_COULOMB = 3
V_RADIAL_SPLINE = 4

# Parity sectors (projectors printed in Sec. 3 beside Fig. 1).
S_NONE = 0
S_PLUS = 1      # P^+
S_MINUS = 2     # P^-
S_PK1 = 3       # P^-_{p_1}
S_PK2 = 4       # P^-_{p_2}
S_PK3 = 5       # P^-_{p_3}

PREC_C64 = 0
PREC_C128 = 1

SCHEME_SPLIT = 0   # FFT kinetic terms: symmetric split-operator step
SCHEME_AB = 1      # FFT kinetic terms: the legacy A/B update with H_K^(1..3)


def smooth_even_sizes(lo: int = 32, hi: int = 256) -> List[int]:
    """Even N in [lo, hi] whose only prime factors are 2, 3 and 5."""
    out = []
    for n in range(lo, hi + 1):
        if n % 2:
            continue
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def initial_states(N: int, k: int, seed: int) -> np.ndarray:
    """k independent complex Gaussian-noise wavefunctions, shape [k, N, N, N].

    Real and imaginary parts are i.i.d. N(0, 1).  Unnormalised: both sides
    orthonormalise before the first step.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((k, N, N, N), dtype=np.complex128)
    n3 = N * N * N
    for i in range(k):
        re = rng.standard_normal(n3)
        im = rng.standard_normal(n3)
        out[i] = (re + 1j * im).reshape(N, N, N)
    return out


# Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
# SC 2011): a counter-based generator.  Ten rounds of two 32 x 32 -> 64-bit multiplies; the
# key is bumped by two Weyl constants between rounds.
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of counters (arrays or scalars of uint32 values) under key (k0, k1);
    returns the four output words as uint64 arrays holding 32-bit values."""
    m = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & m for x in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(k0) & m, np.uint64(k1) & m
    for _ in range(10):
        p0 = np.uint64(PHILOX_M0) * c[0]
        p1 = np.uint64(PHILOX_M1) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & m, p1 & m, ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & m, p0 & m]
        k0 = (k0 + np.uint64(PHILOX_W0)) & m
        k1 = (k1 + np.uint64(PHILOX_W1)) & m
    return c


def philox_noise_states(N: int, k: int, seed: int) -> np.ndarray:
    """k complex Gaussian-noise wavefunctions [k, N, N, N] from Philox4x32-10, the same numbers as
    the library's qfdtd_set_state_noise: site x (C order) of state i uses counter
    (x mod 2^32, x div 2^32, i, 0) and key (seed mod 2^32, seed div 2^32); the words w0..w3 give
    u1 = ((w0 2^21 + w1 div 2^11) + 1) 2^-53 and u2 likewise from w2, w3, both in (0, 1], and
    Re + i Im = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2) (Box-Muller)."""
    n3 = N * N * N
    x = np.arange(n3, dtype=np.uint64)
    out = np.empty((k, N, N, N), dtype=np.complex128)
    for i in range(k):
        w = philox4x32_10(x & np.uint64(0xFFFFFFFF), x >> np.uint64(32), np.full(n3, i, np.uint64),
                          np.zeros(n3, np.uint64), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
        a = ((w[0] << np.uint64(21)) | (w[1] >> np.uint64(11))) + np.uint64(1)
        b = ((w[2] << np.uint64(21)) | (w[3] >> np.uint64(11))) + np.uint64(1)
        u1 = a.astype(np.float64) * 2.0 ** -53
        u2 = b.astype(np.float64) * 2.0 ** -53
        r = np.sqrt(-2.0 * np.log(u1))
        out[i] = (r * np.cos(2 * np.pi * u2) + 1j * r * np.sin(2 * np.pi * u2)).reshape(N, N, N)
    return out


def orbit_uniform_field(N: int, seed: int, lo: float, hi: float,
                        reflect_axes: Sequence[Sequence[int]] = ((0, 1), (2,))) -> np.ndarray:
    """Real field drawn U(lo, hi) once per orbit of a group of reflections.

    The group is generated by the reflections listed in ``reflect_axes``; a
    reflection of axis l maps i_l -> (N - i_l) mod N.  The default group
    {1, R12, R3, R12 R3} is the one under which P^+ and P^-_{p_3} commute with
    a potential; one U(lo, hi) draw per site is made in C order and every site
    takes the draw of its orbit's smallest linear index.  Returns float64
    [N, N, N].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(lo, hi, size=N * N * N).reshape(N, N, N)
    idx = np.arange(N * N * N, dtype=np.int64).reshape(N, N, N)
    rep = idx.copy()
    mirror = (-np.arange(N)) % N
    # close the orbit under the generators (two rounds suffice for 2 commuting involutions)
    gens = []
    for axes in reflect_axes:
        sl = [np.arange(N)] * 3
        for ax in axes:
            sl[ax] = mirror
        gens.append(tuple(sl))
    for _ in range(len(gens)):
        for g in gens:
            moved = rep[np.ix_(*g)]
            rep = np.minimum(rep, moved)
    return u.reshape(-1)[rep.reshape(-1)].reshape(N, N, N)


def spline_knots(L: float, seed: int, n_knots: int = 16) -> np.ndarray:
    """Knots (r_j, V_j) of a smooth random radial potential, shape [n_knots, 2].

    r_j = j R / (n-1) with R = sqrt(3) L / 2 (the lattice corner distance),
    V_j = r_j^2 / 2 + 0.5 u_j, u_j ~ U(-1, 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    R = math.sqrt(3.0) * L / 2.0
    r = np.arange(n_knots, dtype=np.float64) * (R / (n_knots - 1))
    u = rng.uniform(-1.0, 1.0, size=n_knots)
    return np.stack([r, 0.5 * r * r + 0.5 * u], axis=1)


@dataclasses.dataclass
class Problem:
    """One solve: lattice, kinetic term, potential, states and schedule."""
    N: int
    a: float
    m: float
    kinetic: int
    vkind: int
    vparams: tuple = ()
    knots: Optional[np.ndarray] = None        # [n, 2] for V_RADIAL_SPLINE
    vgrid_seed: Optional[int] = None          # imaginary perturbation seed
    vgrid_range: tuple = (0.0, 0.01)
    k: int = 3
    sectors: Optional[tuple] = None
    precision: int = PREC_C64
    dt: float = 0.0
    steps: int = 0
    measure_every: int = 50
    seed: int = 0
    label: str = ""
    scheme: int = 0                           # FFT kinetic terms: 0 split operator, 1 A/B update
    grid: Optional[np.ndarray] = None         # [N, N, N] V of a V_GRID problem

    def init_states(self) -> np.ndarray:
        return initial_states(self.N, self.k, self.seed)

    def v_add_grid(self) -> Optional[np.ndarray]:
        """Additive complex grid (i * perturbation) or None."""
        if self.vgrid_seed is None:
            return None
        lo, hi = self.vgrid_range
        return 1j * orbit_uniform_field(self.N, self.vgrid_seed, lo, hi)

    def abi_grid(self) -> Optional[np.ndarray]:
        """The grid handed to the C ABI: the full V for V_GRID (plus any perturbation), else the
        additive perturbation or None."""
        add = self.v_add_grid()
        if self.vkind == V_GRID:
            g = np.asarray(self.grid, dtype=np.complex128)
            return g if add is None else g + add
        return add


def anisotropic_ho_grid(N: int, a: float, omegas=(1.0, 1.3, 1.7)) -> np.ndarray:
    """V = sum_l omega_l^2 x_l^2 / 2 on the lattice (x_l = (i_l - N/2) a), a V_GRID input whose
    lowest levels are non-degenerate."""
    x = (np.arange(N, dtype=np.float64) - N // 2) * a
    w1, w2, w3 = omegas
    return (0.5 * (w1 * w1 * x[:, None, None] ** 2 + w2 * w2 * x[None, :, None] ** 2
                   + w3 * w3 * x[None, None, :] ** 2)).astype(np.complex128)


HBARC_GEV_FM = 0.1973269804   # hbar c, converts GeV to fm^-1


def coulomb_problem(kinetic: int, N: int = 64, a: float = 0.12, alpha: float = 1.0,
                    sectors: tuple = (S_PLUS, S_PLUS, S_PK3), precision: int = PREC_C64,
                    tau: float = 80.0, K: int = 50, seed: int = 106) -> Problem:
    """Coulomb validation workload (Sec. 3): V = -alpha/r_f (r_f = max(r, a/2)), lattice
    spacing a in fm, reduced mass 0.3 GeV; the paper prints no coupling, alpha = 1 puts the
    Bohr radius 1/(m alpha) = 0.66 fm at 5.5 sites of a = 0.12 fm.  Units: fm and fm^-1;
    dt = m a^2 / 6 (half the H_K^(0) bound); tau = steps * dt."""
    m = 0.3 / HBARC_GEV_FM
    dt = m * a * a / 6.0
    return Problem(N=N, a=a, m=m, kinetic=kinetic, vkind=V_COULOMB, vparams=(alpha, a / 2),
                   k=len(sectors), sectors=tuple(sectors), precision=precision, dt=dt,
                   steps=int(round(tau / dt)), measure_every=K, seed=seed,
                   label="coulomb%d_k%d" % (N, kinetic))


def config1() -> Problem:
    a = 0.25
    return Problem(N=32, a=a, m=1.0, kinetic=K_NR_P2, vkind=V_HARMONIC, vparams=(1.0,),
                   k=3, precision=PREC_C128, dt=a * a / 8, steps=3000, seed=101,
                   label="ho32_p2_c128")


def config2(kinetic: int) -> Problem:
    a = 0.25
    assert kinetic in (K_FDTD, K_NR_SIN2)
    return Problem(N=128, a=a, m=1.0, kinetic=kinetic, vkind=V_HARMONIC, vparams=(1.0,),
                   k=3, precision=PREC_C64, dt=a * a / 8, steps=5000, seed=102,
                   label="ho128_%s_c64" % ("fdtd" if kinetic == K_FDTD else "sin2"))


def config3() -> Problem:
    a = 0.05
    return Problem(N=256, a=a, m=1.5, kinetic=K_REL, vkind=V_CORNELL,
                   vparams=(0.4, 0.2, a / 2), vgrid_seed=1031, k=3,
                   sectors=(S_PLUS, S_PLUS, S_PK3), precision=PREC_C64,
                   dt=a / 8, steps=10000, seed=103, label="cornell256_rel_c64")


BATCH_SIZES = (48, 64, 80, 96, 128, 160)


def config4(n: int = 64, seed: int = 104) -> List[Problem]:
    """Batch of uneven Cornell solves; kinetic kinds split as evenly as possible."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = rng.choice(np.array(BATCH_SIZES), size=n)
    alpha = rng.uniform(0.2, 0.6, size=n)
    sigma = rng.uniform(0.1, 0.3, size=n)
    m = rng.uniform(1.0, 5.0, size=n)
    kinds = np.array([K_NR_P2, K_NR_SIN2, K_REL] * ((n + 2) // 3))[:n]
    rng.shuffle(kinds)
    a = 0.05
    out = []
    for i in range(n):
        out.append(Problem(N=int(Ns[i]), a=a, m=float(m[i]), kinetic=int(kinds[i]),
                           vkind=V_CORNELL, vparams=(float(alpha[i]), float(sigma[i]), a / 2),
                           k=3, precision=PREC_C64, dt=a / 8, steps=5000,
                           seed=seed * 1000 + i, label="batch%02d" % i))
    return out


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after trace start
    problem: Problem


def config5(n_requests: int = 1000, rate: float = 200.0, seed: int = 105,
            precision: int = PREC_C64) -> List[Request]:
    """Poisson stream of single-state solves on tabulated radial potentials."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.array(smooth_even_sizes(32, 256))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ns = rng.choice(sizes, size=n_requests)
    kinds = rng.choice(np.array([K_NR_P2, K_NR_SIN2, K_REL]), size=n_requests)
    out = []
    for j in range(n_requests):
        N = int(Ns[j])
        a = 8.0 / N
        knots = spline_knots(8.0, seed * 100000 + j)
        p = Problem(N=N, a=a, m=1.0, kinetic=int(kinds[j]), vkind=V_RADIAL_SPLINE,
                    knots=knots, k=1, precision=precision, dt=0.01, steps=50000,
                    measure_every=50, seed=seed * 1000000 + j, label="req%04d" % j)
        out.append(Request(rid=j, arrival=float(arrivals[j]), problem=p))
    return out
