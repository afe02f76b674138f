"""Pins of the oracle's BC1 encoder (E1).

The paper fixes the BTC palette and the index rule (Sec. III-A), not the
endpoint search, so the encoder is pinned by what the format and the
mathematics fix:
  * constant blocks reach the optimum of a brute force over all 2^32
    endpoint pairs (and a per-channel error of at most 1 for any colour);
  * two-colour blocks with RGB565-exact colours reach SSE 0; other tiny
    blocks never beat the brute force and the gap is small;
  * the reported SSE equals the SSE of decoding the emitted bits;
  * it is never worse than a plain bounding-box encoder written here.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
from conftest import random_blocks, rgba, smooth_blocks


def _brute(cols, counts):
    lib = O._load()
    f = lib.ref_bc1_bruteforce
    f.restype = ctypes.c_uint64
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    c = np.ascontiguousarray(cols, np.int32)
    n = np.ascontiguousarray(counts, np.int32)
    return int(f(c.ctypes.data, n.ctypes.data, len(n)))


def _sse(tex, blocks):
    dec = O.bc1_decode(blocks).astype(int)
    return ((dec[..., :3] - tex[..., :3].astype(int)) ** 2).sum(axis=(1, 2))


def _const_block(col):
    return rgba(np.tile(np.array(col, np.uint8), (1, 16, 1)))


@pytest.mark.slow
@pytest.mark.parametrize("col", [(37, 201, 90), (3, 130, 250)])
def test_constant_block_is_bruteforce_optimal(col):
    blk, sse = O.bc1_encode(_const_block(col))
    assert int(sse[0]) == _brute([col], [16])


def test_constant_blocks_error_at_most_one_per_channel():
    rng = np.random.default_rng(3)
    cols = rng.integers(0, 256, (4000, 3))
    tex = rgba(np.repeat(cols[:, None, :], 16, 1))
    blocks, sse = O.bc1_encode(tex)
    dec = O.bc1_decode(blocks).astype(int)
    assert np.abs(dec[..., :3] - tex[..., :3].astype(int)).max() <= 1
    assert np.array_equal(sse, _sse(tex, blocks))
    # colours whose channels are all 565 expansions are reproduced exactly
    e5 = lambda c: (c << 3) | (c >> 2)
    e6 = lambda c: (c << 2) | (c >> 4)
    exact = np.array([[e5(r), e6(g), e5(b)] for r, g, b in rng.integers(0, [32, 64, 32], (500, 3))])
    tex = rgba(np.repeat(exact[:, None, :], 16, 1))
    assert O.bc1_encode(tex)[1].max() == 0


def test_two_exact_colours_reach_zero():
    rng = np.random.default_rng(5)
    e5 = lambda c: (c << 3) | (c >> 2)
    e6 = lambda c: (c << 2) | (c >> 4)
    tex = []
    for _ in range(300):
        a = [e5(rng.integers(32)), e6(rng.integers(64)), e5(rng.integers(32))]
        b = [e5(rng.integers(32)), e6(rng.integers(64)), e5(rng.integers(32))]
        sel = rng.integers(0, 2, 16)
        tex.append([a if s else b for s in sel])
    tex = rgba(np.array(tex))
    assert O.bc1_encode(tex)[1].max() == 0


@pytest.mark.slow
def test_two_colour_block_against_bruteforce():
    a, b = (10, 200, 33), (90, 120, 250)
    tex = rgba(np.array([[a] * 9 + [b] * 7]))
    sse = int(O.bc1_encode(tex)[1][0])
    opt = _brute([a, b], [9, 7])
    assert sse >= opt
    assert sse <= opt + 16 * 12   # the gap is reported; it stays small


def test_reported_sse_matches_decode():
    for tex in (random_blocks(600, 11), smooth_blocks(1500, 12), smooth_blocks(500, 13, spread=2)):
        blocks, sse = O.bc1_encode(tex)
        assert np.array_equal(sse, _sse(tex, blocks))


def _bbox_encode_sse(tex):
    """Plain bounding-box BC1 encoder: c0 = max corner, c1 = min corner,
    each texel takes its best palette entry."""
    out = []
    for t in tex[..., :3].astype(int):
        hi, lo = t.max(0), t.min(0)
        q = lambda v: [int(round(v[0] * 31 / 255)), int(round(v[1] * 63 / 255)), int(round(v[2] * 31 / 255))]
        a, b = q(hi), q(lo)
        c0 = a[0] << 11 | a[1] << 5 | a[2]
        c1 = b[0] << 11 | b[1] << 5 | b[2]
        if c0 < c1:
            c0, c1 = c1, c0
        blk = np.array([c0 & 255, c0 >> 8, c1 & 255, c1 >> 8, 0, 0, 0, 0], np.uint8)
        pal = O.bc1_decode(np.array([blk[0], blk[1], blk[2], blk[3], 0xE4, 0xE4, 0xE4, 0xE4], np.uint8))[0, :4, :3].astype(int)
        d = ((t[:, None, :] - pal[None]) ** 2).sum(-1)
        out.append(int(d.min(1).sum()))
    return np.array(out)


def test_never_worse_than_bounding_box():
    tex = np.concatenate([random_blocks(300, 21), smooth_blocks(300, 22)])
    _, sse = O.bc1_encode(tex)
    assert (sse.astype(int) <= _bbox_encode_sse(tex)).all()


def test_refinement_never_hurts():
    tex = smooth_blocks(800, 31, spread=30)
    s0 = O.bc1_encode(tex, refine_steps=0)[1]
    s2 = O.bc1_encode(tex, refine_steps=2)[1]
    assert (s2 <= s0).all() and (s2 < s0).any()


def test_block_layout():
    """c0/c1 little-endian 565 words, then 2-bit indices, texel 0 lowest; a
    4-colour block has c0 > c1."""
    tex = smooth_blocks(200, 41, spread=40)
    blocks, _ = O.bc1_encode(tex)
    c0 = blocks[:, 0].astype(int) | blocks[:, 1].astype(int) << 8
    c1 = blocks[:, 2].astype(int) | blocks[:, 3].astype(int) << 8
    assert (c0 > c1).mean() > 0.5


def _angle(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    c = abs(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
    return float(np.arccos(min(1.0, c)))


def test_principal_axis_special_cases():
    """E1 step 2: no spread gives (1, 1, 1); spread in one channel only gives
    that channel's axis; collinear texels give their line."""
    assert O.principal_axis(np.full((16, 3), 77)).tolist() == [1, 1, 1]
    x = np.zeros((16, 3), np.int32)
    x[:, 1] = np.arange(16) * 13
    v = O.principal_axis(x)
    assert v[0] == 0 and v[2] == 0 and v[1] != 0
    d = np.array([3, -5, 7])
    x = 120 + np.outer(np.arange(-8, 8), d)
    assert _angle(O.principal_axis(x), d) < 1e-3


def test_principal_axis_matches_the_dominant_eigenvector():
    """On random point clouds with a clear dominant direction (eigenvalue
    ratio below 1/2), eight integer power steps land within a few
    milliradians of numpy's top eigenvector of the covariance."""
    rng = np.random.default_rng(31)
    done = 0
    while done < 300:
        n = int(rng.integers(3, 17))
        d = rng.normal(size=3)
        t = rng.normal(size=n) * rng.uniform(10, 60)
        x = np.clip(np.rint(128 + np.outer(t, d / np.linalg.norm(d)) + rng.normal(size=(n, 3)) * rng.uniform(0, 12)),
                    0, 255).astype(np.int32)
        w, V = np.linalg.eigh(np.cov(x.T.astype(np.float64), bias=True))
        if w[2] <= 0 or w[1] / w[2] > 0.5:
            continue
        assert _angle(O.principal_axis(x), V[:, 2]) < 0.01, (x.tolist(), w.tolist())
        done += 1
