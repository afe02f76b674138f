"""CPU checks of integer identities the BC1 kernel relies on.

The cluster fit divides by the determinant of each split's 2x2 normal
equations with a 32-bit multiply-high: floor(n / det) = floor(n M / 2^36),
M = ceil(2^36 / det), for every dividend the kernel can form (below
512 det).  Checked here exhaustively for every determinant of the 4- and
3-cluster split lists."""
import numpy as np


def _split_dets():
    dets = set()
    for four in (0, 1):
        for s1 in range(17):
            for s2 in range(s1, 17):
                for s3 in (range(s2, 17) if four else [16]):
                    n0, n1, n2, n3 = s1, s2 - s1, s3 - s2, 16 - s3
                    A = 9 * n0 + 4 * n1 + n2 if four else 4 * n0 + n1
                    B = n1 + 4 * n2 + 9 * n3 if four else n1 + 4 * n2
                    AB = 2 * (n1 + n2) if four else n1
                    d = A * B - AB * AB
                    assert d >= 0
                    if d:
                        dets.add(d)
    return sorted(dets)


def test_split_determinants_fit_the_multiplier():
    dets = _split_dets()
    assert min(dets) >= 1 and max(dets) <= 2 ** 13
    for d in dets:
        M = ((1 << 36) + d - 1) // d
        assert M < 2 ** 32


def test_multiply_high_division_is_exact():
    for d in _split_dets():
        M = np.uint64(((1 << 36) + d - 1) // d)
        n = np.arange(0, 512 * d, dtype=np.uint64)
        hi = (n * M) >> np.uint64(32)                 # the 32-bit multiply-high
        assert np.array_equal(hi >> np.uint64(4), n // np.uint64(d)), d
