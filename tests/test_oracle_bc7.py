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


def _ls_reference(x, idx, nb):
    """Endpoints by numpy's least squares on the stacked design matrix
    (rows (64 - w, w), targets 64 x), rounded half up with exact fractions
    deciding values within 1e-6 of a half, clamped to [0, 255]."""
    from fractions import Fraction
    m = (1 << nb) - 1
    w = np.array([(128 * k + m) // (2 * m) for k in idx], np.int64)
    D = np.stack([64 - w, w], 1).astype(np.float64)
    if np.linalg.matrix_rank(D) < 2:
        return None
    sol, *_ = np.linalg.lstsq(D, 64.0 * x.astype(np.float64), rcond=None)   # [2][nch]
    A, B, AB = int(((64 - w) ** 2).sum()), int((w * w).sum()), int(((64 - w) * w).sum())
    det = A * B - AB * AB
    out = np.empty_like(sol, dtype=np.int64)
    for e in range(2):
        for c in range(sol.shape[1]):
            v = sol[e, c]
            if abs(v - np.floor(v) - 0.5) < 1e-6:                 # a possible tie: decide exactly
                SA, SB = int(((64 - w) * x[:, c]).sum()), int((w * x[:, c]).sum())
                num = 64 * (B * SA - AB * SB) if e == 0 else 64 * (A * SB - AB * SA)
                v = Fraction(num, det)
                out[e, c] = int(np.floor(v + Fraction(1, 2)))
            else:
                out[e, c] = int(np.floor(v + 0.5))
    return np.clip(out, 0, 255)


@pytest.mark.parametrize("nb", [2, 3, 4])
def test_least_squares_refit_matches_lstsq(nb):
    """E2 step (d): the refit endpoints equal an independent least-squares
    solve of (64 - w) e0 + w e1 = 64 x, rounded half up and clamped, on
    random members (1 to 16, RGB and one channel), ties included; a single
    used index (singular system) gives no refit."""
    rng = np.random.default_rng(40 + nb)
    for trial in range(400):
        n = int(rng.integers(1, 17))
        nch = 3 if trial % 4 else 1
        x = rng.integers(0, 256, (n, nch))
        if trial % 7 == 0:
            x[:] = x[0]                                            # equal members: exact ties likely
        idx = rng.integers(0, 1 << nb, n)
        got = O.bc7_ls_endpoints(x, idx, nb)
        ref = _ls_reference(x, idx, nb)
        if ref is None:
            assert got is None
            continue
        assert got is not None
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (trial, x.tolist(), idx.tolist())
    assert O.bc7_ls_endpoints(np.array([[5, 6, 7], [9, 9, 9]]), [1, 1], 2) is None
