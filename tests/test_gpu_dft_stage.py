"""The DFT-stage measurement library on the GPU: both variants compute the 16-point DFT.

Each variant against a direct FP64 evaluation of the DFT sum on the host, for the forward
transform (reps = 1), the round trip (reps = 2, forward then inverse / 16) and three stages.
FP32 tolerance: the stage error grows like log2(16) ulp for the butterfly and like sqrt(16)
ulp for the dense product; 1e-6 of the largest output bounds both.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def dft16(x, sign=-1):
    j = np.arange(16)
    F = np.exp(sign * 2j * np.pi * np.outer(j, j) / 16)
    return x @ F.T


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("reps", [1, 2, 3])
def test_dft16_stage_matches_the_dft_sum(variant, reps):
    import torch
    from paper_2211_10185_amd import dft_stage as D
    print("dft16 stage variant=%s reps=%d" % (variant, reps), flush=True)
    rng = np.random.default_rng(5 + reps)
    nvec = 512
    x = (rng.standard_normal((nvec, 16)) + 1j * rng.standard_normal((nvec, 16))).astype(np.complex64)
    y = D.run(torch.from_numpy(x).cuda(), reps, variant).cpu().numpy().astype(np.complex128)
    ref = x.astype(np.complex128)
    for r in range(reps):
        ref = dft16(ref) if r % 2 == 0 else dft16(ref, +1) / 16
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    assert err < 1e-6, err


def test_dft16_stage_rejects_bad_sizes():
    import torch
    from paper_2211_10185_amd import dft_stage as D
    x = torch.zeros(100, 16, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        D.run(x, 1, "valu")
