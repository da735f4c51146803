"""Host input generators: the Philox4x32-10 definition against the published
known-answer vectors (Random123 distribution of Salmon, Moraes, Dror and
Shaw, SC 2011), and the Box-Muller normals it feeds."""
import numpy as np

from paper_2110_09841_amd import synth

# (counter, key) -> output, all words hexadecimal
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        got = synth.philox4x32_10(np.array([ctr]), key)[0]
        assert tuple(int(v) for v in got) == want


def test_philox_gaussian_moments_and_layout():
    n = 400003
    z = synth.philox_gaussian(n, seed=0x0123456789ABCDEF)
    assert z.shape == (n,)
    # N(0,1): mean within 5 standard errors, variance within 5 standard errors
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    # fourth moment of a normal is 3
    assert abs((z ** 4).mean() - 3.0) < 0.05
    # the draws for a prefix do not depend on n (counter-based)
    assert np.array_equal(synth.philox_gaussian(9, seed=0x0123456789ABCDEF), z[:9])
    # different seeds give different streams
    assert not np.allclose(synth.philox_gaussian(16, seed=1), synth.philox_gaussian(16, seed=2))
