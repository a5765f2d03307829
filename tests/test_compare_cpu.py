"""The sampled L2 estimator used against the stored oracle results, checked on the CPU."""
import numpy as np

from compare import phase_aligned_l2, sampled_state_errors, subspace_distance


def _setup(seed, n3=18 ** 3, k=3, eps=1e-5):
    rng = np.random.default_rng(seed)
    ref = rng.standard_normal((k, n3)) + 1j * rng.standard_normal((k, n3))
    ref, _ = np.linalg.qr(ref.T)
    ref = ref.T
    pert = eps * (rng.standard_normal((k, n3)) + 1j * rng.standard_normal((k, n3)))
    dens = (np.abs(ref) ** 2).mean(0)
    dens /= dens.sum()
    q = 0.5 / n3 + 0.5 * dens
    sites = rng.choice(n3, size=4096, p=q)
    return rng, ref, pert, q, sites


def test_sampled_estimate_tracks_the_exact_phase_aligned_l2():
    rng, ref, pert, q, sites = _setup(1)
    gpu = (ref + pert) * np.exp(1j * rng.uniform(0, 6.28, size=(3, 1)))
    est = sampled_state_errors(gpu[:, sites], ref[:, sites], q[sites], [0.0, 1.0, 2.0])
    exact = np.array([phase_aligned_l2(gpu[i], ref[i]) for i in range(3)])
    assert np.all(np.abs(est / exact - 1) < 0.15), (est, exact)


def test_sampled_estimate_of_a_degenerate_pair_is_its_subspace_distance():
    rng, ref, pert, q, sites = _setup(2)
    U, _ = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
    gpu = ref + pert
    gpu[1:] = U @ gpu[1:]                   # any basis of the degenerate pair
    est = sampled_state_errors(gpu[:, sites], ref[:, sites], q[sites], [0.0, 1.0, 1.0])
    d = subspace_distance(gpu[1:], ref[1:])
    assert d < 2e-3                          # the perturbation only
    assert np.all(np.abs(est[1:] / d - 1) < 0.3), (est, d)
    # without the degeneracy the same rotation is a large per-state error
    est2 = sampled_state_errors(gpu[:, sites], ref[:, sites], q[sites], [0.0, 1.0, 2.0])
    assert est2[1] > 0.1
