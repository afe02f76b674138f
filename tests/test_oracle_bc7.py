"""Pins of the oracle's BC7 encoder (E2).

  * every constant RGB block is reproduced exactly (mode 5 reaches every
    8-bit value at weights 21 and 43, so SSE 0 is always attainable);
  * the reported SSE equals the SSE of the emitted bits decoded by Pillow
    (an independent decoder), so every field, p-bit and anchor rule is laid
    out as the format requires;
  * the full search is never worse than any single-mode search, and a
    single-mode search emits only that mode;
  * blocks of two colours exactly representable in mode 6 reach SSE 0.
"""
import numpy as np
import pytest

import oracle as O
from conftest import random_blocks, rgba, smooth_blocks

PIL = pytest.importorskip("PIL.Image")


def _pillow(blocks):
    im = PIL.frombytes("RGBA", (4 * blocks.shape[0], 4), blocks.tobytes(), "bcn", 7)
    a = np.asarray(im)
    return a.reshape(4, blocks.shape[0], 4, 4).transpose(1, 0, 2, 3).reshape(blocks.shape[0], 16, 4)


def _mode(b0):
    return next(m for m in range(8) if (b0 >> m) & 1)


def _rgb_sse(tex, dec):
    return ((dec[..., :3].astype(int) - tex[..., :3].astype(int)) ** 2).sum(axis=(1, 2))


def test_candidate_enumeration():
    seen = [O.bc7_candidate(i) for i in range(285)]
    assert [m for m, *_ in seen].count(0) == 16
    for m in (1, 2, 3, 7):
        assert sorted(p for mm, p, _, _ in seen if mm == m) == list(range(64))
    assert sorted((r, s) for m, _, r, s in seen if m == 4) == [(r, s) for r in range(4) for s in range(2)]
    assert sorted(r for m, _, r, _ in seen if m == 5) == [0, 1, 2, 3]
    with pytest.raises(IndexError):
        O.bc7_candidate(285)


def test_constant_blocks_exact():
    greys = np.repeat(np.arange(256)[:, None], 3, 1)
    rng = np.random.default_rng(7)
    cols = np.concatenate([greys, rng.integers(0, 256, (1500, 3))])
    tex = rgba(np.repeat(cols[:, None, :], 16, 1))
    blocks, sse = O.bc7_encode(tex)
    assert sse.max() == 0
    assert np.array_equal(_pillow(blocks)[..., :3], tex[..., :3])


def test_sse_matches_independent_decode():
    for tex in (random_blocks(150, 1), smooth_blocks(400, 2), smooth_blocks(200, 3, spread=3)):
        blocks, sse = O.bc7_encode(tex)
        assert np.array_equal(sse, _rgb_sse(tex, _pillow(blocks)))
        assert np.array_equal(O.bc7_decode(blocks), _pillow(blocks))


def test_every_mode_alone_is_valid_and_full_search_wins():
    tex = np.concatenate([smooth_blocks(60, 4, spread=20), random_blocks(30, 5)])
    full = O.bc7_encode(tex)[1]
    for m in range(8):
        blocks, sse = O.bc7_encode(tex, mode_mask=1 << m)
        assert all(_mode(int(b)) == m for b in blocks[:, 0])
        assert np.array_equal(sse, _rgb_sse(tex, _pillow(blocks)))
        assert (full <= sse).all()


def test_mode6_exact_pairs_reach_zero():
    rng = np.random.default_rng(9)
    tex = []
    for _ in range(200):
        pa, pb = rng.integers(0, 2, 2)
        a = rng.integers(0, 128, 3) * 2 + pa      # one p-bit per endpoint
        b = rng.integers(0, 128, 3) * 2 + pb
        sel = rng.integers(0, 2, 16)
        tex.append([a if s else b for s in sel])
    blocks, sse = O.bc7_encode(rgba(np.array(tex)))
    assert sse.max() == 0


def test_bc7_beats_bc1_on_smooth_blocks():
    tex = smooth_blocks(300, 8)
    s1 = O.bc1_encode(tex)[1].astype(np.int64).sum()
    s7 = O.bc7_encode(tex)[1].astype(np.int64).sum()
    assert s7 < s1
