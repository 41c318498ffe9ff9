"""Host checks of the integer identities the tiled sweeps rely on.

* The tile of a cell: for every tile extent d the library accepts (1..64
  cells) and every cell coordinate c of a tiled grid (at most 1024 cells per
  axis), floor(c / d) equals (c * ceil(2^16 / d)) >> 16, and the product fits
  the 24-bit multiplier's operands and a 32-bit result.
* The global cell index c0 + n0 (c1 + n1 c2): with n0, n1 <= 1024 every
  factor fed to a 24-bit multiply is below 2^24 and the index below 2^30.
* The moves left inside a tile per axis are below 64, so three of them pack
  into ten-bit fields of one 32-bit word without carries between fields.
"""
import numpy as np


def test_tile_quotient_by_reciprocal_multiply():
    c = np.arange(1024, dtype=np.int64)
    for d in range(1, 65):
        m = (65536 + d - 1) // d
        assert m < 1 << 24 and int(c.max()) * m < 1 << 32
        assert np.array_equal((c * m) >> 16, c // d), d


def test_reciprocal_multiply_fails_beyond_the_accepted_extents():
    # the identity is not general: it breaks for larger divisors, which the
    # library rejects (tile extents above 64 cells)
    c = np.arange(1024, dtype=np.int64)
    bad = [d for d in range(65, 1025) if not np.array_equal((c * ((65536 + d - 1) // d)) >> 16, c // d)]
    assert bad and min(bad) > 64


def test_global_index_factors_fit_24_bits():
    n = 1024
    inner = (n - 1) + n * (n - 1)  # c1 + n1 c2 at its largest
    assert n < 1 << 24 and inner < 1 << 24
    assert (n - 1) + n * inner < 1 << 30


def test_moves_left_pack_without_carries():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        r = rng.integers(0, 64, size=3)
        rp = int(r[0]) | int(r[1]) << 10 | int(r[2]) << 20
        # a move decrements one non-zero field
        a = int(rng.integers(0, 3))
        if r[a] == 0:
            continue
        rp -= 1 << (10 * a)
        r[a] -= 1
        assert [(rp >> (10 * k)) & 1023 for k in range(3)] == [int(v) for v in r]
