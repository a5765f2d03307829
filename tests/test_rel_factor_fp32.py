"""Accuracy of the complex64 path's relativistic k-space factor against the FP64 symbol.

In complex64 the factor exp(-dt T3(k)) / N^3 of eq. HK3 (rest mass removed,
T3 = sqrt(p^2 + m^2) - m) is evaluated per site in FP32 from a per-axis table of
lattice momenta squared, p_l^2 = 4 sin^2(k_l/2)/a^2 (FP64-generated, stored in
FP32).  T3 enters only the exponent, so the cancellation in sqrt(p^2 + m^2) - m
costs at most dt sqrt(p^2 + m^2) 2^-24 in absolute terms.  This test evaluates
that FP32 formula with correctly rounded FP32 operations over the whole grids of
the relativistic workloads and bounds its relative error against the FP64
factor; the GPU uses single-instruction sqrt and 2^x, each within about 1 ulp,
which adds at most a few ulp more (the GPU test of the applied factor checks
that).  The A/B update's factor is dt T3 itself; there the kernels use
p^2 / (sqrt(p^2 + m^2) + m), which has no cancellation.
"""
import numpy as np

import oracle as O


def fp32_factor(N, a, m, dt):
    """exp(-dt T3) / N^3 by the kernel's FP32 formula, per axis table -> [N, N, N]."""
    f32 = np.float32
    # 4 sin^2(k/2)/a^2 per axis: the H_K^(2) symbol with 2M = 1 along axis 1 (k2 = k3 = 0)
    kt = O.kinetic_symbol(O.K_NR_SIN2, N, a, 0.5)[:, 0, 0].astype(f32)
    p2 = (kt[:, None, None] + kt[None, :, None]) + kt[None, None, :]
    mm = f32(m)
    tk = np.sqrt(p2 + mm * mm) - mm
    c = (-f32(dt)) * f32(1.4426950408889634)
    return np.exp2(c * tk) * f32(1.0 / N ** 3)


def test_fp32_relativistic_factor_error_bound_at_256():
    p_N, a, m, dt = 256, 0.05, 1.5, 0.05 / 8
    want = np.exp(-dt * O.kinetic_symbol(O.K_REL, p_N, a, m)) / p_N ** 3
    got = fp32_factor(p_N, a, m, dt).astype(np.float64)
    rel = np.abs(got - want) / want
    worst = float(rel.max())
    print("max relative error of the FP32 factor over 256^3:", worst)
    # FP32 rounding of the table, three adds, sqrt, the subtraction, two products and 2^x: a
    # few units of 2^-24 = 6.0e-8, with the exponent error scaled by dt sqrt(p^2 + m^2) <= 0.43
    assert worst < 6e-7
    # dt T3 at the Nyquist corner, the largest exponent
    assert abs(dt * (np.sqrt(12 / a ** 2 + m * m) - m) - 0.4235) < 1e-3


def test_fp32_relativistic_factor_error_bound_on_the_batch_and_serving_shapes():
    # the other relativistic workloads: batch members (a = 0.05, dt = a/8, m up to 5) and
    # serving requests (a = 8/N, dt = 0.01, m = 1) at their largest sizes
    for N, a, m, dt in [(160, 0.05, 5.0, 0.05 / 8), (256, 8 / 256, 1.0, 0.01), (144, 8 / 144, 1.0, 0.01)]:
        want = np.exp(-dt * O.kinetic_symbol(O.K_REL, N, a, m)) / N ** 3
        got = fp32_factor(N, a, m, dt).astype(np.float64)
        worst = float((np.abs(got - want) / want).max())
        print("N", N, "a", a, "m", m, "dt", dt, "max relative error", worst)
        assert worst < 6e-7
