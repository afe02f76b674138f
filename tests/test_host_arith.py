"""CPU checks of arithmetic identities the encoders rely on.

BC1: the cluster fit divides by the determinant of each split's 2x2 normal
equations with a 32-bit multiply-high: floor(n / det) = floor(n M / 2^36),
M = ceil(2^36 / det), for every dividend the kernel can form (below
512 det).  Checked here exhaustively for every determinant of the 4- and
3-cluster split lists.

BC7: the least-squares refit's FP64 rounding (below)."""
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


# ---------------------------------------------------------------------------
# BC7 least-squares refit (Sec. III-B): endpoint e0 = round-half-up of
# 64 (B SA - AB SB) / det, clamped to [0, 255], with A = sum (64 - w)^2,
# B = sum w^2, AB = sum (64 - w) w, SA = sum (64 - w) x, SB = sum w x over a
# subset's members.  The kernel forms the numerator exactly in FP64 (scaled
# by -8), takes 1/det from the FP32 hardware reciprocal refined by two FP64
# Newton steps, and rounds floor(m inv + 1/2 + 2^-37).  The hardware
# reciprocal is within 1 ulp; here it is modelled as the correctly rounded
# FP32 reciprocal moved by -2..+2 ulp, every FP64 fused multiply-add rounded
# once from its exact value, and the result compared with the exact
# rational floor.
from fractions import Fraction

_HALF_MARGIN = 0.5 + 2.0 ** -37


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _inverse(det, ulps):
    """-8/det as the kernel computes it, from a reciprocal `ulps` units off."""
    r = np.float32(1.0) / np.float32(det)
    toward = np.float32(np.inf) if ulps > 0 else np.float32(0.0)
    for _ in range(abs(ulps)):
        r = np.nextafter(r, toward, dtype=np.float32)
    inv = float(r)
    inv = _fma(_fma(-det, inv, 1.0), inv, inv)
    return -8.0 * _fma(_fma(-det, inv, 1.0), inv, inv)


def _refit_cases(rng, nb, count):
    """Member sets the kernel can present: 1..16 members, NB-bit indices with
    the format's weights, 8-bit texels; plus exact half-way cases."""
    wts = [(128 * i + (1 << nb) - 1) // (2 * ((1 << nb) - 1)) for i in range(1 << nb)]
    cases = []
    for _ in range(count):
        n = int(rng.integers(2, 17))
        w = [wts[int(i)] for i in rng.integers(0, 1 << nb, n)]
        x = rng.integers(0, 256, (n, 3)).tolist()
        if rng.random() < 0.2:   # saturated texels
            x = [[int(v) for v in rng.choice([0, 255], 3)] for _ in range(n)]
        cases.append((w, x))
    # endpoint = mean of the texels at one end: ties at exactly .5, .25, .75
    for n0 in (2, 4):
        for s in range(0, 4 * 255 + 1, 37):
            xs = [min(255, s // n0 + (k < s % n0)) for k in range(n0)]
            if sum(xs) != s:
                continue
            cases.append(([0] * n0 + [64] * 3, [[v, 255 - v, v // 2] for v in xs] + [[7, 250, 128]] * 3))
    return cases


def _exact(N, det):
    return min(255, max(0, (128 * N + det) // (2 * det)))


def test_bc7_refit_rounding_with_perturbed_reciprocal():
    rng = np.random.default_rng(20260)
    checked = 0
    for nb in (2, 3, 4):
        for w, x in _refit_cases(rng, nb, 400):
            n = len(w)
            W1, W2 = sum(w), sum(v * v for v in w)
            A, B, AB = 4096 * n - 128 * W1 + W2, W2, 64 * W1 - W2
            det = A * B - AB * AB
            if det == 0:
                continue
            assert 0 < det < 2 ** 32
            invs = [_inverse(float(det), u) for u in (-2, -1, 0, 1, 2)]
            for c in range(3):
                SA = sum((64 - wi) * xi[c] for wi, xi in zip(w, x))
                SB = sum(wi * xi[c] for wi, xi in zip(w, x))
                # the kernel's -8-scaled sums and numerators (exact in FP64)
                SA8, SB8 = -8 * SA, -8 * SB
                m0, m1 = B * SA8 - AB * SB8, A * SB8 - AB * SA8
                assert abs(m0) < 2 ** 53 and abs(m1) < 2 ** 53
                e0, e1 = _exact(B * SA - AB * SB, det), _exact(A * SB - AB * SA, det)
                for inv in invs:
                    q0, q1 = _fma(float(m0), inv, _HALF_MARGIN), _fma(float(m1), inv, _HALF_MARGIN)
                    assert int(min(max(q0, 0.0), 255.0)) == e0, (nb, w, x, c)
                    assert int(min(max(q1, 0.0), 255.0)) == e1, (nb, w, x, c)
                    checked += 1
    assert checked > 15000


def test_bc7_refit_half_way_quotients():
    """Half-way endpoints: with weights 0 and 64 only, e0 is the mean S0 / n0
    of the n0 texels at weight 0, so sums with S0 / n0 = k + 1/2 put
    64 N / det + 1/2 exactly on an integer, with determinants 2^24 n0 n64
    that are not powers of two (every third sum, each reciprocal offset)."""
    checked = 0
    for n0, n64 in ((2, 1), (2, 3), (4, 3), (6, 5), (8, 7), (10, 3), (14, 1)):
        w = [0] * n0 + [64] * n64
        n, W1, W2 = len(w), sum(w), sum(v * v for v in w)
        A, B, AB = 4096 * n - 128 * W1 + W2, W2, 64 * W1 - W2
        det = A * B - AB * AB
        assert AB == 0 and det == 4096 * 4096 * n0 * n64
        invs = [_inverse(float(det), u) for u in (-2, -1, 0, 1, 2)]
        for S0 in range(1, 255 * n0, 3):
            N = B * 64 * S0                      # SA = 64 S0, AB = 0
            e = _exact(N, det)
            assert e == min(255, (2 * S0 + n0) // (2 * n0))
            for inv in invs:
                assert int(min(max(_fma(float(-8 * N), inv, _HALF_MARGIN), 0.0), 255.0)) == e, (n0, n64, S0)
                checked += 1
    assert checked > 19000
