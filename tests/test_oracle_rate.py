"""Pins of the oracle's rate controller (R): exact bit budget, and the greedy
choice equals a brute force over every subset of upgraded bands."""
import itertools

import numpy as np
import pytest

import oracle as O
from conftest import smooth_blocks


def _rand_sse(rng):
    s7 = rng.integers(10_000, 2_000_000, 16)
    s1 = s7 + rng.integers(0, 3_000_000, 16)
    vmin = -rng.uniform(0.01, 1.0, 16).astype(np.float32)
    vmax = rng.uniform(0.01, 1.0, 16).astype(np.float32)
    return s1.astype(np.int64), s7.astype(np.int64), vmin, vmax


@pytest.mark.parametrize("rate", [4.25 + 0.25 * k for k in range(16)])
def test_exact_budget(rate):
    rng = np.random.default_rng(int(rate * 4))
    s1, s7, vmin, vmax = _rand_sse(rng)
    fmt = O.rate_select(s1, s7, vmin, vmax, rate)
    assert fmt[0] == 7
    nblk = 1234
    bits = sum(nblk * (64 if f == 1 else 128) for f in fmt)
    assert bits == rate * 16 * (nblk * 16)


@pytest.mark.parametrize("rate", [4.0, 4.3, 6.1, 8.25, 9.0, -1.0])
def test_infeasible_rates(rate):
    rng = np.random.default_rng(3)
    assert O.rate_select(*_rand_sse(rng), rate) is None


def test_greedy_equals_bruteforce():
    """Minimising the coefficient-domain error sum_k E_k(format) * delta_k^2
    over every subset of k upgraded bands gives the oracle's choice."""
    rng = np.random.default_rng(4)
    for trial in range(30):
        s1, s7, vmin, vmax = _rand_sse(rng)
        rate = 4.25 + 0.25 * int(rng.integers(0, 16))
        k = int(4 * rate - 17)
        fmt = O.rate_select(s1, s7, vmin, vmax, rate)
        d2 = np.array([float(np.float32((vmax[b] - vmin[b]) / np.float32(255.0))) ** 2 for b in range(16)])
        best, best_set = None, None
        for sub in itertools.combinations(range(1, 16), k):
            err = sum((s7[b] if b in sub else s1[b]) * d2[b] for b in range(1, 16))
            if best is None or err < best:
                best, best_set = err, sub
        assert set(np.nonzero(fmt[1:] == 7)[0] + 1) == set(best_set)


def test_encode_auto_round_trip():
    rng = np.random.default_rng(6)
    nblk = 40
    tex = np.stack([smooth_blocks(nblk, 100 + b, spread=2 + 3 * b) for b in range(16)])
    vmin = np.full(16, -0.5, np.float32)
    vmax = np.full(16, 0.5, np.float32)
    payload, off, fmt = O.encode_auto(tex, vmin, vmax, 6.0)
    assert (fmt == 7).sum() == 8 and fmt[0] == 7
    dec = O.decode_stream(payload, off, fmt, nblk)
    for b in range(16):
        if fmt[b] == 7:
            assert np.array_equal(dec[b], O.bc7_decode(O.bc7_encode(tex[b])[0]))
        else:
            assert np.array_equal(dec[b], O.bc1_decode(O.bc1_encode(tex[b])[0]))
    assert O.encode_auto(tex, vmin, vmax, 6.1) is None
