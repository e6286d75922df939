"""The observation digest used by the whole-population parity tests: the
oracle library's C sum equals the numpy definition, and the mistakes a
placement bug makes (a changed byte, two bytes swapped, two values shifted
in opposite directions) change it."""
import numpy as np

import oracle as O
from digest import digest_numpy, weights

BLOCK = 48800


def test_weights_are_splitmix64():
    # SplitMix64 (Steele, Lea and Flood 2014) from state 0: its first outputs
    w = weights(3)
    assert [int(x) for x in w] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_c_digest_equals_the_numpy_definition():
    rng = np.random.default_rng(0)
    for block in (1, 100, BLOCK):
        x = rng.integers(0, 256, size=(13, block), dtype=np.uint8)
        assert np.array_equal(O.digest_blocks(x, block), digest_numpy(x))


def test_digest_sees_placement_mistakes():
    rng = np.random.default_rng(1)
    x = (rng.random((1, BLOCK)) < 0.02).astype(np.uint8) * rng.integers(1, 256, size=(1, BLOCK), dtype=np.uint8)
    base = O.digest_blocks(x, BLOCK)[0]
    nz = np.flatnonzero(x[0])
    y = x.copy()
    y[0, nz[3]] ^= 1                                  # one byte changed
    assert O.digest_blocks(y, BLOCK)[0] != base
    y = x.copy()
    i, j = nz[5], nz[5] + 7
    y[0, i], y[0, j] = x[0, j], x[0, i]               # two bytes swapped
    assert x[0, i] != x[0, j] and O.digest_blocks(y, BLOCK)[0] != base
    y = np.zeros_like(x)
    y[0, 1000], y[0, 5000] = 1, 1
    z = np.zeros_like(x)
    z[0, 1001], z[0, 4999] = 1, 1                     # opposite one-square shifts
    assert O.digest_blocks(y, BLOCK)[0] != O.digest_blocks(z, BLOCK)[0]
