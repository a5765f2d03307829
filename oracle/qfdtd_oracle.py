"""FP64 CPU oracle for the imaginary-time Schroedinger evolution.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
path (the HIP library and its Python binding) never calls it and shares no code
with it; both sides take their seeded inputs from ``synthetic``.

Everything here is plain numpy in complex128 / float64, written from the paper
(arXiv:2211.10185, "QuantumFDTD - A computational framework for the relativistic
Schroedinger equation"):

* Hamiltonian split H = H_K + V                                  (Sec. 2, eq. eq_schro)
* kinetic terms H_K^(0) .. H_K^(3)                              (Sec. 2, eqs. HK0-HK3)
* lattice momenta k_l = A p_l, Nyquist +pi kept                  (Sec. 2, text after HK3)
* imaginary-time evolution -d/dtau Psi = H Psi, decaying modes   (Sec. 2, eq. eq_iterat and
                                                                  the general solution after it)
* excited states by orthogonal projection                        (Sec. 1)
* parity projectors P^+, P^-, P^-_{p_k}                          (Sec. 3, beside Fig. 1)

A library FFT (scipy.fft, unnormalised forward, 1/N^3 on the inverse) serves as
the transform step.  No blocking, fusion or reordering beyond the definitions
below: each imaginary-time step is applied to each state in full.

Readings of the paper that this oracle takes (the text is silent or ambiguous):

* The update rule is deferred to the cited legacy code.  FFT kinetic terms use
  the symmetric split-operator step  psi <- h * IFFT[exp(-dt T) FFT[h psi]],
  h = exp(-dt V / 2).  H_K^(0) uses the legacy explicit form with the potential
  averaged over the step: psi <- A psi - B dt H_K^(0) psi,
  A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2).
* The same legacy form with H_K^(0) swapped for an FFT kinetic term (the paper
  changes only the kinetic operator of the legacy iteration) is the second
  scheme, SCHEME_AB: psi <- A psi - B dt IFFT[T FFT[psi]].  It is stable for
  dt <= 2 / max T (``ab_dt_bound``).
* The printed H_K^(0) carries 1/(2A) * 1/A per neighbour difference; this
  oracle uses the standard 7-point Laplacian over A^2 (the paper states that
  H_K^(0) and H_K^(1,2) agree away from the walls, which needs that factor).
* The evolution equation is read with the full H = H_K + V.
* H_K^(3) is evolved and reported with the rest mass removed: T - M.
* The origin is on site N/2 (x_l = (i_l - N/2) a); FDTD walls are ghost zeros
  at i_l = -1 and i_l = N.
* Excited states: k states evolve together and are re-orthonormalised by
  modified Gram-Schmidt (per parity sector, in state order) every K steps and
  after the last step.
* P^-_{p_k} uses the idempotent normalisation 1/4 (the printed 1/2 only
  rescales, which normalisation removes).
* On the walled lattice a site with some i_l = 0 has its mirror image on the
  wall, so a state of definite parity vanishes there; the projectors set those
  sites to zero (which keeps them idempotent).
* Energies are Rayleigh quotients <psi_i|H|psi_i> of the normalised states.
"""
from __future__ import annotations

import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.fft as sfft
from scipy.interpolate import CubicSpline

WORKERS = int(os.environ.get("QFDTD_ORACLE_THREADS", os.cpu_count() or 1))

K_FDTD, K_NR_P2, K_NR_SIN2, K_REL = 0, 1, 2, 3
V_GRID, V_HARMONIC, V_CORNELL, V_COULOMB, V_RADIAL_SPLINE = 0, 1, 2, 3, 4
S_NONE, S_PLUS, S_MINUS, S_PK1, S_PK2, S_PK3 = 0, 1, 2, 3, 4, 5
SCHEME_SPLIT, SCHEME_AB = 0, 1


# --------------------------------------------------------------------------
# lattice geometry and potentials
# --------------------------------------------------------------------------

def coords(N: int, a: float) -> np.ndarray:
    """x_l = (i_l - N/2) a for i_l = 0..N-1 (origin on site N/2)."""
    return (np.arange(N, dtype=np.float64) - N // 2) * a


def radius(N: int, a: float) -> np.ndarray:
    x = coords(N, a)
    return np.sqrt(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)


def potential(N: int, a: float, vkind: int, vparams: Sequence[float] = (),
              knots: Optional[np.ndarray] = None, grid: Optional[np.ndarray] = None,
              add_grid: Optional[np.ndarray] = None) -> np.ndarray:
    """V(r) on the lattice as complex128 [N, N, N].

    Harmonic: V = k r^2 / 2.  Cornell: V = -alpha / r_f + sigma r_f with
    r_f = max(r, r_floor).  Coulomb: V = -alpha / r_f.  Radial spline: natural
    cubic spline through the knots (r_j, V_j) evaluated at r.  Grid: the given
    array.  ``add_grid`` is added to any of them (e.g. an imaginary part).
    """
    r = radius(N, a)
    if vkind == V_HARMONIC:
        kk = vparams[0] if len(vparams) else 1.0
        v = 0.5 * kk * r * r
    elif vkind == V_CORNELL:
        alpha, sigma, rf = vparams
        re = np.maximum(r, rf)
        v = -alpha / re + sigma * re
    elif vkind == V_COULOMB:
        alpha, rf = vparams[0], vparams[1]
        v = -alpha / np.maximum(r, rf)
    elif vkind == V_RADIAL_SPLINE:
        cs = CubicSpline(knots[:, 0], knots[:, 1], bc_type="natural")
        v = cs(r)
    elif vkind == V_GRID:
        v = np.asarray(grid)
    else:
        raise ValueError("unknown potential kind %r" % vkind)
    v = np.asarray(v, dtype=np.complex128)
    if add_grid is not None:
        v = v + add_grid
    return v


# --------------------------------------------------------------------------
# kinetic terms
# --------------------------------------------------------------------------

def lattice_momenta(N: int) -> np.ndarray:
    """k for FFT index j: j' = j if j <= N/2 else j - N, k = 2 pi j' / N.

    This is the set {-pi + 2pi/N, ..., 0, ..., pi} of Sec. 2 in FFT order.
    """
    j = np.arange(N)
    jp = np.where(j <= N // 2, j, j - N)
    return 2.0 * np.pi * jp / N


def kinetic_symbol(kind: int, N: int, a: float, m: float) -> np.ndarray:
    """T(k) on the FFT grid, float64 [N, N, N] (eqs. HK1, HK2, HK3).

    HK1: sum k_l^2 / (2 M A^2).   HK2: 4 sum sin^2(k_l/2) / (2 M A^2).
    HK3: sqrt(4 sum sin^2(k_l/2) / A^2 + M^2) - M  (the 1/(A N^3) prefactor of
    eq. HK3 is A^-1 sqrt(A^2 p^2 + (AM)^2) with the 1/N^3 of the inverse FFT).
    """
    k = lattice_momenta(N)
    k1, k2, k3 = k[:, None, None], k[None, :, None], k[None, None, :]
    if kind == K_NR_P2:
        return (k1 ** 2 + k2 ** 2 + k3 ** 2) / (2.0 * m * a * a)
    s = 4.0 * (np.sin(k1 / 2) ** 2 + np.sin(k2 / 2) ** 2 + np.sin(k3 / 2) ** 2)
    if kind == K_NR_SIN2:
        return s / (2.0 * m * a * a)
    if kind == K_REL:
        return np.sqrt(s / (a * a) + m * m) - m
    raise ValueError("no FFT symbol for kinetic kind %r" % kind)


def fft3(psi: np.ndarray) -> np.ndarray:
    """Unnormalised forward 3D DFT, sum_x psi(x) exp(-i k.x)."""
    return sfft.fftn(psi, axes=(-3, -2, -1), workers=WORKERS)


def ifft3(phi: np.ndarray) -> np.ndarray:
    """Inverse 3D DFT including the 1/N^3 factor."""
    return sfft.ifftn(phi, axes=(-3, -2, -1), workers=WORKERS)


def laplacian_dirichlet(psi: np.ndarray) -> np.ndarray:
    """L_D psi(i) = sum over the 6 neighbours psi(i +- e_l) - 6 psi(i), psi = 0 outside [0, N)."""
    p = np.pad(psi, 1)
    c = p[1:-1, 1:-1, 1:-1]
    return (p[2:, 1:-1, 1:-1] + p[:-2, 1:-1, 1:-1] + p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1]
            + p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] - 6.0 * c)


def apply_kinetic(psi: np.ndarray, kind: int, a: float, m: float,
                  T: Optional[np.ndarray] = None) -> np.ndarray:
    """H_K psi for any of the four kinetic terms."""
    if kind == K_FDTD:
        return -laplacian_dirichlet(psi) / (2.0 * m * a * a)
    if T is None:
        T = kinetic_symbol(kind, psi.shape[-1], a, m)
    return ifft3(T * fft3(psi))


def apply_hamiltonian(psi, kind, a, m, V, T=None):
    return apply_kinetic(psi, kind, a, m, T) + V * psi


# --------------------------------------------------------------------------
# closed forms of the continuum Coulomb problem (validation references, Sec. 3)
# --------------------------------------------------------------------------

def hydrogen_level(n: int, m: float, alpha: float) -> float:
    """E_n = -m alpha^2 / (2 n^2) of H = p^2/(2m) - alpha/r."""
    return -m * alpha * alpha / (2.0 * n * n)


def hydrogen_state(name: str, N: int, a: float, m: float, alpha: float) -> np.ndarray:
    """Continuum 1s, 2s or 2p_z (along x3) wavefunction sampled at the lattice sites, with the
    continuum normalisation (a^3 sum |psi|^2 -> 1); Bohr radius a_B = 1/(m alpha)."""
    aB = 1.0 / (m * alpha)
    r = radius(N, a)
    if name == "1s":
        return np.exp(-r / aB) / np.sqrt(np.pi * aB ** 3)
    if name == "2s":
        return (2.0 - r / aB) * np.exp(-r / (2 * aB)) / np.sqrt(32 * np.pi * aB ** 3)
    if name == "2p":
        z = coords(N, a)[None, None, :]
        return (z / aB) * np.exp(-r / (2 * aB)) / np.sqrt(32 * np.pi * aB ** 3)
    raise ValueError(name)


def hydrogen_1s_momentum(p: np.ndarray, m: float, alpha: float) -> np.ndarray:
    """1s wavefunction in momentum space (wavenumber p, int |phi|^2 d^3p = 1):
    phi(p) = 2 sqrt(2) a_B^{3/2} / (pi (1 + a_B^2 p^2)^2); the radial diagnostic of Sec. 3 is
    y(p) = sqrt(4 pi) p phi(p)."""
    aB = 1.0 / (m * alpha)
    return 2.0 * np.sqrt(2.0) * aB ** 1.5 / (np.pi * (1.0 + (aB * p) ** 2) ** 2)


# --------------------------------------------------------------------------
# one imaginary-time step
# --------------------------------------------------------------------------

def split_factors(T: np.ndarray, V: np.ndarray, dt: float):
    """The two factors of the symmetric split step: h = exp(-dt V / 2) and exp(-dt T)."""
    return np.exp(-0.5 * dt * V), np.exp(-dt * T)


def step_split(psi: np.ndarray, T: np.ndarray, V: np.ndarray, dt: float,
               factors=None) -> np.ndarray:
    """Symmetric split step  h IFFT[exp(-dt T) FFT[h psi]],  h = exp(-dt V / 2).

    ``factors`` may carry ``split_factors(T, V, dt)`` computed once for many steps; the
    values are the same either way."""
    h, eT = split_factors(T, V, dt) if factors is None else factors
    return h * ifft3(eT * fft3(h * psi))


def step_ab_fft(psi: np.ndarray, T: np.ndarray, V: np.ndarray, dt: float) -> np.ndarray:
    """psi <- A psi - B dt H_K psi with H_K psi = IFFT[T FFT[psi]] (the legacy update, FFT kinetic term)."""
    A = (1.0 - 0.5 * dt * V) / (1.0 + 0.5 * dt * V)
    B = 1.0 / (1.0 + 0.5 * dt * V)
    return A * psi - B * dt * ifft3(T * fft3(psi))


def ab_dt_bound(kind: int, a: float, m: float) -> float:
    """Largest stable dt of the A/B update: dt * max T <= 2 (max T at k = (pi, pi, pi))."""
    if kind == K_FDTD or kind == K_NR_SIN2:
        tmax = 6.0 / (m * a * a)
    elif kind == K_NR_P2:
        tmax = 3.0 * np.pi ** 2 / (2.0 * m * a * a)
    else:
        tmax = np.sqrt(12.0 / (a * a) + m * m) - m
    return 2.0 / tmax


def step_fdtd(psi: np.ndarray, V: np.ndarray, dt: float, a: float, m: float) -> np.ndarray:
    """psi <- A psi + B dt L_D psi / (2 M A^2), A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2)."""
    A = (1.0 - 0.5 * dt * V) / (1.0 + 0.5 * dt * V)
    B = 1.0 / (1.0 + 0.5 * dt * V)
    return A * psi + B * (dt / (2.0 * m * a * a)) * laplacian_dirichlet(psi)


def step_fdtd_at(psi: np.ndarray, V_at: np.ndarray, dt: float, a: float, m: float,
                 sites: np.ndarray) -> np.ndarray:
    """The H_K^(0) update of ``step_fdtd`` at the given sites only ([n, 3] indices; V_at the
    potential there), from the six neighbours of each site (zero beyond the walls).  For
    lattices too large to step whole."""
    N = psi.shape[0]
    i1, i2, i3 = sites[:, 0], sites[:, 1], sites[:, 2]

    def at(j1, j2, j3):
        ok = (j1 >= 0) & (j1 < N) & (j2 >= 0) & (j2 < N) & (j3 >= 0) & (j3 < N)
        out = np.zeros(len(sites), dtype=np.complex128)
        out[ok] = psi[j1[ok], j2[ok], j3[ok]]
        return out

    c = at(i1, i2, i3)
    lap = (at(i1 + 1, i2, i3) + at(i1 - 1, i2, i3) + at(i1, i2 + 1, i3) + at(i1, i2 - 1, i3)
           + at(i1, i2, i3 + 1) + at(i1, i2, i3 - 1) - 6.0 * c)
    A = (1.0 - 0.5 * dt * V_at) / (1.0 + 0.5 * dt * V_at)
    B = 1.0 / (1.0 + 0.5 * dt * V_at)
    return A * c + B * (dt / (2.0 * m * a * a)) * lap


# --------------------------------------------------------------------------
# parity projectors and Gram-Schmidt
# --------------------------------------------------------------------------

def reflect(psi: np.ndarray, axes: Sequence[int], periodic: bool = True) -> np.ndarray:
    """(psi o R)(i) = psi(R i), R_l : i_l -> N - i_l (mod N on the periodic lattice).

    With the origin on site N/2 this is x_l -> -x_l.  On the Dirichlet lattice the
    image of i_l = 0 is the wall (N), where psi = 0.
    """
    out = psi
    N = psi.shape[-1]
    src = (-np.arange(N)) % N
    for ax in axes:
        out = np.take(out, src, axis=ax)       # a new array
        if not periodic:
            sl = [slice(None)] * out.ndim
            sl[ax] = 0
            out[tuple(sl)] = 0.0
    return out


def parity_project(psi: np.ndarray, sector: int, periodic: bool = True) -> np.ndarray:
    """P^+ = (1 + R)/2,  P^- = (1 - R)/2,  P^-_{p_k} = (1 + R_{other two})(1 - R_k)/4.

    On the walled lattice only the sites with every i_l >= 1 have their mirror image inside
    the box (the mirror of i_l = 0 is the wall, where psi = 0), so a state of definite parity
    vanishes wherever some i_l = 0; the projection sets those sites to zero.  This keeps the
    walled projectors idempotent and the sectors orthogonal (Sec. 3 uses them as projectors).
    """
    if sector == S_NONE:
        return psi
    if sector in (S_PLUS, S_MINUS):
        sgn = 1.0 if sector == S_PLUS else -1.0
        out = 0.5 * (psi + sgn * reflect(psi, (0, 1, 2), periodic))
    else:
        kax = sector - S_PK1
        others = tuple(ax for ax in (0, 1, 2) if ax != kax)
        out = 0.25 * (psi + reflect(psi, others, periodic) - reflect(psi, (kax,), periodic)
                      - reflect(psi, (0, 1, 2), periodic))
    if not periodic:
        out[0, :, :] = 0.0
        out[:, 0, :] = 0.0
        out[:, :, 0] = 0.0
    return out


def inner(x: np.ndarray, y: np.ndarray) -> complex:
    """Lattice inner product sum conj(x) y."""
    return complex(np.vdot(x.ravel(), y.ravel()))


def gram_schmidt(states: List[np.ndarray], sectors: Sequence[int]) -> List[np.ndarray]:
    """Modified Gram-Schmidt in state order; states in different sectors are not mixed."""
    out: List[np.ndarray] = []
    for i, psi in enumerate(states):
        v = psi.copy()
        for j in range(i):
            if sectors[j] == sectors[i]:
                v = v - inner(out[j], v) * out[j]
        v = v / np.sqrt(inner(v, v).real)
        out.append(v)
    return out


# --------------------------------------------------------------------------
# measurement and the whole iteration
# --------------------------------------------------------------------------

def energies(states: Sequence[np.ndarray], kind: int, a: float, m: float,
             V: np.ndarray, T: Optional[np.ndarray] = None) -> np.ndarray:
    """E_i = <psi_i|H|psi_i> / <psi_i|psi_i> (complex when V is complex)."""
    if kind != K_FDTD and T is None:
        T = kinetic_symbol(kind, states[0].shape[-1], a, m)
    out = []
    for psi in states:
        hp = apply_hamiltonian(psi, kind, a, m, V, T)
        out.append(inner(psi, hp) / inner(psi, psi).real)
    return np.array(out, dtype=np.complex128)


def project_and_orthonormalise(states, sectors, periodic):
    states = [parity_project(s, sec, periodic) for s, sec in zip(states, sectors)]
    return gram_schmidt(states, sectors)


def evolve(states: List[np.ndarray], kind: int, a: float, m: float, V: np.ndarray,
           dt: float, steps: int, K: int, sectors: Sequence[int],
           trace: Optional[list] = None, scheme: int = SCHEME_SPLIT,
           map_fn=map) -> List[np.ndarray]:
    """Run ``steps`` steps in chunks of K; project + orthonormalise after each chunk.

    ``states`` must already be projected and orthonormalised (see ``prepare``).
    If ``trace`` is a list, the energies after every chunk are appended to it.
    ``scheme`` selects the step of the FFT kinetic terms (split operator or A/B).
    ``map_fn`` applies one step to every state; the states are independent between two
    orthonormalisations, so a thread pool's ``map`` gives the same results as ``map``.
    """
    periodic = kind != K_FDTD
    T = kinetic_symbol(kind, states[0].shape[-1], a, m) if periodic else None
    fac = split_factors(T, V, dt) if periodic and scheme == SCHEME_SPLIT else None
    done = 0
    while done < steps:
        n = min(K, steps - done)
        for _ in range(n):
            if periodic and scheme == SCHEME_AB:
                states = list(map_fn(lambda s: step_ab_fft(s, T, V, dt), states))
            elif periodic:
                states = list(map_fn(lambda s: step_split(s, T, V, dt, fac), states))
            else:
                states = list(map_fn(lambda s: step_fdtd(s, V, dt, a, m), states))
        done += n
        states = project_and_orthonormalise(states, sectors, periodic)
        if trace is not None:
            trace.append(energies(states, kind, a, m, V, T))
    return states


def prepare(init: np.ndarray, sectors: Sequence[int], periodic: bool) -> List[np.ndarray]:
    """Project the initial states onto their sectors and orthonormalise them."""
    return project_and_orthonormalise([np.asarray(s, dtype=np.complex128) for s in init],
                                      sectors, periodic)


def problem_potential(p) -> np.ndarray:
    """V for a ``synthetic.Problem``."""
    return potential(p.N, p.a, p.vkind, p.vparams, knots=p.knots, grid=getattr(p, "grid", None),
                     add_grid=p.v_add_grid())


def solve(p, steps: Optional[int] = None, init: Optional[np.ndarray] = None,
          trace: Optional[list] = None) -> Dict[str, object]:
    """Full oracle solve of a ``synthetic.Problem``: energies and states in state order."""
    steps = p.steps if steps is None else steps
    sectors = list(p.sectors) if p.sectors else [S_NONE] * p.k
    V = problem_potential(p)
    init = p.init_states() if init is None else init
    periodic = p.kinetic != K_FDTD
    states = prepare(init, sectors, periodic)
    states = evolve(states, p.kinetic, p.a, p.m, V, p.dt, steps, p.measure_every, sectors,
                    trace, getattr(p, "scheme", SCHEME_SPLIT))
    E = energies(states, p.kinetic, p.a, p.m, V)
    return {"energies": E, "states": np.stack(states), "sectors": sectors}


def solve_until_converged(p, tol: float = 1e-8, max_steps: Optional[int] = None,
                          init: Optional[np.ndarray] = None) -> Dict[str, object]:
    """Single-state serving rule: stop when |E0(chunk m) - E0(chunk m-1)| < tol."""
    max_steps = p.steps if max_steps is None else max_steps
    sectors = list(p.sectors) if p.sectors else [S_NONE] * p.k
    V = problem_potential(p)
    periodic = p.kinetic != K_FDTD
    T = kinetic_symbol(p.kinetic, p.N, p.a, p.m) if periodic else None
    states = prepare(p.init_states() if init is None else init, sectors, periodic)
    prev = None
    done = 0
    E = None
    while done < max_steps:
        states = evolve(states, p.kinetic, p.a, p.m, V, p.dt, p.measure_every,
                        p.measure_every, sectors, None, getattr(p, "scheme", SCHEME_SPLIT))
        done += p.measure_every
        E = energies(states, p.kinetic, p.a, p.m, V, T)
        if prev is not None and abs(E[0] - prev) < tol:
            break
        prev = E[0]
    return {"energies": E, "states": np.stack(states), "steps": done}


# --------------------------------------------------------------------------
# snapshot extraction of excited states (the legacy method, Sec. 1)
# --------------------------------------------------------------------------

def snapshot_run(p, steps: int, every: int, init: Optional[np.ndarray] = None):
    """Evolve state 0 of ``p`` alone, normalised every ``every`` steps; the normalised state
    after each chunk is a snapshot.  Returns (snapshots [n][N,N,N], taus [n])."""
    V = problem_potential(p)
    periodic = p.kinetic != K_FDTD
    init = p.init_states() if init is None else init
    sec = [p.sectors[0]] if p.sectors else [S_NONE]
    st = prepare(init[:1], sec, periodic)
    snaps, taus = [], []
    done = 0
    while done < steps:
        n = min(every, steps - done)
        st = evolve(st, p.kinetic, p.a, p.m, V, p.dt, n, n, sec, None, getattr(p, "scheme", SCHEME_SPLIT))
        done += n
        snaps.append(st[0].copy())
        taus.append(done * p.dt)
    return snaps, np.array(taus)


def snapshot_energies(p, snaps: Sequence[np.ndarray], fixed: Sequence[np.ndarray]):
    """Orthogonal projection of each snapshot against the orthonormal ``fixed`` states (in
    order): returns (E(tau_j), r_j) with r_j the norm of the projected snapshot (the snapshots
    have unit norm) and E(tau_j) the Rayleigh quotient of the projected snapshot."""
    V = problem_potential(p)
    E, r = [], []
    for sj in snaps:
        v = sj.copy()
        for f in fixed:
            v = v - inner(f, v) * f
        nv = np.sqrt(inner(v, v).real)
        r.append(nv)
        with np.errstate(invalid="ignore", divide="ignore"):
            E.append(energies([v / nv], p.kinetic, p.a, p.m, V)[0] if nv > 0 else np.nan)
    return np.array(E), np.array(r)


def stationary_point(E: np.ndarray, r: np.ndarray, floor: float):
    """Where E(tau_j) stops improving: its minimum (real part) over the snapshots whose
    projected norm r_j exceeds ``floor``.  The Rayleigh quotient of a projected snapshot falls
    while the higher levels decay; once r_j nears the rounding of the projection the remainder is
    noise.  Returns (index, value)."""
    e = np.real(np.asarray(E)).astype(np.float64)
    ok = np.isfinite(e) & (np.asarray(r) > floor)
    e = np.where(ok, e, np.inf)
    j = int(np.argmin(e))
    return j, float(e[j])
