"""Comparison metrics for GPU-vs-oracle parity (no method arithmetic here)."""
import numpy as np


def phase_aligned_l2(a, b):
    """min over theta of ||e^{i theta} a - b|| / ||b||."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    ov = np.vdot(a, b)
    ph = ov / abs(ov) if abs(ov) > 0 else 1.0
    return float(np.linalg.norm(a * ph - b) / np.linalg.norm(b))


def subspace_distance(A, B):
    """Largest principal-angle sine between the column spans of A and B."""
    qa, _ = np.linalg.qr(np.asarray(A).reshape(A.shape[0], -1).T)
    qb, _ = np.linalg.qr(np.asarray(B).reshape(B.shape[0], -1).T)
    # ||(I - Qa Qa^H) Qb||_2: accurate for small angles (sqrt(1 - cos^2) is not)
    r = qb - qa @ (qa.conj().T @ qb)
    return float(np.linalg.norm(r, 2))


def energy_errors(E, E_ref):
    """|E - E_ref| / max(|E_ref|, |E_{k-1} - E_0|, 1e-2) per level."""
    E = np.asarray(E)
    E_ref = np.asarray(E_ref)
    spread = float(np.max(E_ref.real) - np.min(E_ref.real)) if len(E_ref) > 1 else 0.0
    den = np.maximum(np.maximum(np.abs(E_ref), spread), 1e-2)
    return np.abs(E - E_ref) / den


def degenerate_clusters(E, tol=1e-6):
    """Groups of state indices whose energies agree within tol * max(1, |E|)."""
    E = np.asarray(E).real
    order = list(range(len(E)))
    groups = []
    for i in order:
        for g in groups:
            if abs(E[g[0]] - E[i]) < tol * max(1.0, abs(E[i])):
                g.append(i)
                break
        else:
            groups.append([i])
    return groups


def wavefunction_errors(psi, psi_ref, E_ref, tol_deg=1e-6):
    """Per-state phase-aligned L2 errors; degenerate clusters use the subspace distance."""
    errs = np.zeros(len(psi_ref))
    for g in degenerate_clusters(E_ref, tol_deg):
        if len(g) == 1:
            errs[g[0]] = phase_aligned_l2(psi[g[0]], psi_ref[g[0]])
        else:
            d = subspace_distance(psi[g], psi_ref[g])
            errs[g] = d
    return errs


def sampled_state_errors(psi_sites, ref_sites, q, E_ref, tol_deg=1e-6):
    """L2 errors of whole-lattice states estimated from their values at sampled sites.

    ``psi_sites``, ``ref_sites``: [k, n] values of the (normalised) states at n sites drawn
    with replacement from the density q ([n], q(x_j) at the sampled sites), so that
    sum_x |f(x)|^2 ~ mean_j |f(x_j)|^2 / q(x_j).  Each state is aligned by the phase that
    minimises the sampled residual; a (near-)degenerate cluster by the unitary that does
    (weighted orthogonal Procrustes), which makes the result the cluster's subspace distance.
    Returns the relative residual per state."""
    psi_sites = np.asarray(psi_sites)
    ref_sites = np.asarray(ref_sites)
    w = 1.0 / (len(q) * np.asarray(q))
    errs = np.zeros(ref_sites.shape[0])
    for g in degenerate_clusters(E_ref, tol_deg):
        A = ref_sites[g]              # [m, n]
        B = psi_sites[g]
        M = (A * w) @ B.conj().T      # sum_j w_j A_j B_j^H, [m, m]
        U, _, Vh = np.linalg.svd(M)
        R = U @ Vh                    # the unitary closest to mapping B onto A
        D = R @ B - A
        for a, i in enumerate(g):
            errs[i] = np.sqrt(np.sum(w * np.abs(D[a]) ** 2) / np.sum(w * np.abs(A[a]) ** 2))
    return errs


def energy_rel_errors(E, E_ref, floor=1e-12):
    """Plain |E - E_ref| / |E_ref| per level (printed beside the spread-normalised metric)."""
    E_ref = np.asarray(E_ref)
    return np.abs(np.asarray(E) - E_ref) / np.maximum(np.abs(E_ref), floor)
