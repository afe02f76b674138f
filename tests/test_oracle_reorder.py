"""Pins of the oracle's quantiser (Q), keys (K), sort (S) and packer (B)."""
import numpy as np

import oracle as O
from paper_2607_14513_amd import synth


def test_quantiser_special_values_and_error_bound():
    pos, sh = synth.make_scene(5000, seed=11)
    sh[:, 7, :] = 0.25                                   # a constant band
    vmin, vmax = O.band_range(sh)
    assert vmin[7] == vmax[7] == np.float32(0.25)
    assert np.array_equal(vmin, sh.min(axis=(0, 2))) and np.array_equal(vmax, sh.max(axis=(0, 2)))
    q = O.quantise(sh, vmin, vmax)
    assert not q[:, 7, :].any()
    for k in range(16):
        if k == 7:
            continue
        band = sh[:, k, :]
        assert q[:, k, :][band == vmin[k]].max() == 0
        assert q[:, k, :][band == vmax[k]].min() == 255
        delta = (float(vmax[k]) - float(vmin[k])) / 255.0
        err = np.abs(float(vmin[k]) + q[:, k, :].astype(np.float64) * delta - band.astype(np.float64))
        # half a step, plus the FP32 rounding of (x - min) * s near 255
        assert err.max() <= (0.5 + 2.0 ** -10) * delta
        # monotone: a larger coefficient never gets a smaller code
        o = np.argsort(band.ravel(), kind="stable")
        assert (np.diff(q[:, k, :].ravel()[o].astype(int)) >= 0).all()


def _interleave_str(r, g, b):
    """Bit interleave by strings: R7 G7 B7 R6 G6 B6 ... R0 G0 B0."""
    rs, gs, bs = (format(v, "08b") for v in (r, g, b))
    return int("".join(rs[i] + gs[i] + bs[i] for i in range(8)), 2)


def test_morton_rgb_matches_string_interleave():
    rng = np.random.default_rng(0)
    cases = [(0, 0, 0), (255, 255, 255), (255, 0, 0), (0, 255, 0), (0, 0, 255), (1, 2, 4), (128, 64, 32)]
    cases += [tuple(int(x) for x in rng.integers(0, 256, 3)) for _ in range(2000)]
    for r, g, b in cases:
        assert O.morton_rgb(r, g, b) == _interleave_str(r, g, b)


def test_zigzag_is_the_textbook_z_order():
    # 4x4 recursive zigzag (Z-order) scan: scan position at each (row, col)
    z = [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
    for y in range(4):
        for x in range(4):
            assert O.zigzag_texel(z[y][x]) == 4 * y + x


def _deinterleave3(m, g):
    c = [0, 0, 0]
    for bit in range(g):
        for a in range(3):
            c[a] |= ((m >> (3 * bit + a)) & 1) << bit
    return c


def test_keys_chunk_and_colour_fields():
    pos, sh = synth.make_scene(3000, seed=12)
    vmin, vmax = O.band_range(sh)
    q = O.quantise(sh, vmin, vmax)
    lo, hi = O.pos_aabb(pos)
    g = 3
    k = O.keys(pos, q, g, lo, hi)
    cells = np.array([_deinterleave3(int(x) >> 24, g) for x in k])
    assert cells.min() == 0 and cells.max() == 2 ** g - 1
    for a in range(3):
        o = np.argsort(pos[:, a], kind="stable")
        assert (np.diff(cells[o, a]) >= 0).all()          # monotone along each axis
        assert cells[np.argmin(pos[:, a]), a] == 0
        assert cells[np.argmax(pos[:, a]), a] == 2 ** g - 1
    for i in range(0, 3000, 37):
        assert int(k[i]) & 0xFFFFFF == _interleave_str(*q[i, 0])
    assert int(k.max()) < (1 << (24 + 3 * g))


def test_sort_is_the_stable_sort():
    rng = np.random.default_rng(2)
    for n in (1, 2, 17, 1000, 50_000):
        k = rng.integers(0, 40, n).astype(np.uint64) << np.uint64(20)
        assert np.array_equal(O.sort(k), np.argsort(k, kind="stable").astype(np.uint32))


def test_pack_is_a_bijection_with_padding():
    for n in (1, 15, 16, 17, 1000):
        rng = np.random.default_rng(n)
        q = rng.integers(0, 256, (n, 16, 3)).astype(np.uint8)
        perm = rng.permutation(n).astype(np.uint32)
        tex = O.pack(q, perm)
        nblk = (n + 15) // 16
        assert tex.shape == (16, nblk, 16, 4)
        assert (tex[..., 3] == 255).all()
        z = [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
        where = {z[y][x]: 4 * y + x for y in range(4) for x in range(4)}
        for s in range(nblk * 16):
            src = perm[min(s, n - 1)]
            assert np.array_equal(tex[:, s // 16, where[s % 16], :3], q[src])


def test_reorder_groups_by_chunk_then_colour():
    pos, sh = synth.make_scene(20_000, seed=13)
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    assert np.array_equal(np.sort(perm), np.arange(20_000))
    q = O.quantise(sh, vmin, vmax)
    lo, hi = O.pos_aabb(pos)
    k = O.keys(pos, q, 3, lo, hi)
    assert (np.diff(k[perm].astype(np.int64)) >= 0).all()


def test_coverage_range_order_statistic():
    """The paper's range (Sec. V-A): the least symmetric [-t, t] holding 99.5 %
    of a band's coefficients.  Built bands with known order statistics: |x|
    a permutation of 1..M with random signs, so t is the rank ceil(0.995 M)."""
    rng = np.random.default_rng(4)
    for n in (1000, 1001, 7):                              # 0.995*3n integer or not
        M = 3 * n
        sh = np.empty((n, 16, 3), np.float32)
        for k in range(16):
            v = rng.permutation(M).astype(np.float32) + 1
            v *= rng.choice([-1.0, 1.0], M).astype(np.float32)
            sh[:, k, :] = (v * (0.25 * (k + 1))).reshape(n, 3)
        vmin, vmax = O.band_range_coverage(sh)
        r = -(-M * 995 // 1000)
        for k in range(16):
            t = np.float32(r * 0.25 * (k + 1))
            assert vmax[k] == t and vmin[k] == -t
            inside = (np.abs(sh[:, k, :]) <= t).mean()
            assert inside >= 0.995 and (np.abs(sh[:, k, :]) < t).mean() < 0.995


def test_coverage_range_zero_band_and_quantisation():
    pos, sh = synth.make_scene(2000, seed=12)
    sh[:, 4, :] = 0.0
    vmin, vmax = O.band_range_coverage(sh)
    assert vmin[4] == 0.0 and vmax[4] == 0.0 and not np.signbit(vmin[4])
    q = O.quantise(sh, vmin, vmax)
    assert not q[:, 4, :].any()
    for k in (0, 1, 9):
        band = sh[:, k, :]
        inside = np.abs(band) <= vmax[k]
        assert inside.mean() >= 0.995
        # values outside the interval clamp to the ends; 0 maps to the middle code
        hi, lo = band >= vmax[k], band <= vmin[k]
        assert hi.any() and q[:, k, :][hi].min() == 255
        assert not lo.any() or q[:, k, :][lo].max() == 0
        assert int(O.quantise(np.zeros((1, 16, 3), np.float32), vmin, vmax)[0, k, 0]) in (127, 128)


def test_premultiply_is_the_fp32_product():
    pos, sh = synth.make_scene(500, seed=13)
    rng = np.random.default_rng(5)
    mu = rng.uniform(0, 1, 500).astype(np.float32)
    mu[:3] = (0.0, 1.0, 0.5)
    h = O.premultiply(sh, mu)
    assert np.array_equal(h, (mu[:, None, None] * sh).astype(np.float32))
    assert not h[0].any() and np.array_equal(h[1], sh[1]) and np.array_equal(h[2], sh[2] * np.float32(0.5))
    # mu = 1 everywhere: reorder unchanged; a power-of-two opacity scales the coverage range exactly
    a = O.reorder(pos, sh, quantiser=1)
    b = O.reorder(pos, sh, quantiser=1, opacity=np.ones(500, np.float32))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    c = O.reorder(pos, sh, quantiser=1, opacity=np.full(500, 0.25, np.float32))
    assert np.array_equal(c[3], a[3] * np.float32(0.25))
