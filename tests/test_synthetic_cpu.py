"""The seeded input generators: Philox4x32-10 against its published known-answer vectors."""
import numpy as np

import synthetic as S


def test_philox4x32_10_known_answers():
    # the known-answer vectors of the generator's reference distribution (Salmon et al., SC 2011)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for c, k, want in cases:
        got = S.philox4x32_10(*[np.array([x], dtype=np.uint64) for x in c], *k)
        assert tuple(int(w[0]) for w in got) == want


def test_philox_noise_is_standard_complex_gaussian_and_seeded():
    z = S.philox_noise_states(24, 2, 7)
    assert z.shape == (2, 24, 24, 24)
    for part in (z.real, z.imag):
        assert abs(part.mean()) < 0.02 and abs(part.var() - 1) < 0.03
    assert abs(np.mean(z.real * z.imag)) < 0.02
    np.testing.assert_array_equal(z, S.philox_noise_states(24, 2, 7))
    assert not np.allclose(z[0], z[1]) and not np.allclose(z, S.philox_noise_states(24, 2, 8))
