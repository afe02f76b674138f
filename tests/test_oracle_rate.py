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


# ---------------------------------------------------------------------------
# The 0-bit option (Sec. IV-B: a band coded with no bits is dropped and
# decodes to zero).  Band 0 BC7; bands 1..S-1 each BC7 (8 bits/texel), BC1
# (4) or dropped (0); exactly rate*S bits per texel-position.

PREF = (7, 1, 3)           # BC7, BC1, dropped: the order that breaks ties
UNITS = np.array([2, 1, 0])


def _delta(vmin, vmax, b):
    return float(np.float32(np.float32(vmax[b]) - np.float32(vmin[b])) / np.float32(255.0))


def _distortions(s1, s7, tex, vmin, vmax, S, direct=False):
    """D[b] = (BC7, BC1, dropped) in coefficient units.  The dropped band's
    error is the sum of its squared dequantised texel values: from the code
    histogram in code order (the definition's form) or, with direct, summed
    texel by texel (a different rounding of the same quantity)."""
    D = np.zeros((S, 3))
    for b in range(1, S):
        d = _delta(vmin, vmax, b)
        D[b, 0] = float(s7[b]) * (d * d)
        D[b, 1] = float(s1[b]) * (d * d)
        codes = tex[b][..., :3].reshape(-1)
        if direct:
            v = float(vmin[b]) + codes.astype(np.float64) * d
            D[b, 2] = float(np.sum(v * v))
        else:
            h = np.bincount(codes, minlength=256)
            z = 0.0
            for q in range(256):
                v = float(vmin[b]) + q * d
                z += float(h[q]) * (v * v)
            D[b, 2] = z
    return D


def _brute(D, S, U):
    """Every assignment of bands 1..S-1, in order (band 1 most significant,
    BC7 < BC1 < dropped); the first of least objective, the objective summed
    from band S-1 down to band 1."""
    n = S - 1
    if n == 0:
        return np.array([7], np.uint8)
    pow3 = 3 ** np.arange(n - 1, -1, -1)
    total = 3 ** n
    chunk = min(total, 3 ** 10)
    best, best_idx = np.inf, None
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk))
        dig = (idx[:, None] // pow3[None, :]) % 3
        s = np.zeros(len(idx))
        for j in range(n - 1, -1, -1):
            s = D[j + 1][dig[:, j]] + s
        s[UNITS[dig].sum(axis=1) != U] = np.inf
        i = int(np.argmin(s))
        if s[i] < best:
            best, best_idx = s[i], idx[i]
    return np.array([7] + [PREF[d] for d in (best_idx // pow3) % 3], np.uint8)


def _scene(rng, S, nblk=8):
    """Band textures with different spreads and offsets, and per-band ranges;
    the SSEs are drawn so that BC7 < BC1 per band."""
    tex = np.zeros((S, nblk, 16, 4), np.uint8)
    for b in range(S):
        mid = int(rng.integers(20, 236))
        spread = int(rng.integers(1, 40))
        tex[b] = np.clip(mid + rng.integers(-spread, spread + 1, (nblk, 16, 4)), 0, 255)
    s7 = rng.integers(1_000, 400_000, 16).astype(np.int64)
    s1 = s7 + rng.integers(0, 600_000, 16)
    vmin = -rng.uniform(0.001, 0.3, 16).astype(np.float32)
    vmax = rng.uniform(0.001, 0.3, 16).astype(np.float32)
    return tex, s1, s7, vmin, vmax


def _units(rate, S):
    return int(round(rate * S / 4)) - 2


@pytest.mark.parametrize("S", [4, 9])
def test_zero_option_equals_bruteforce(S):
    rng = np.random.default_rng(40 + S)
    for trial in range(12):
        tex, s1, s7, vmin, vmax = _scene(rng, S)
        for U in range(0, 2 * (S - 1) + 1):
            rate = (U + 2) * 4 / S
            fmt = O.rate_select_zero(s1, s7, O.band_hist(tex), vmin, vmax, rate, S)
            want = _brute(_distortions(s1, s7, tex, vmin, vmax, S), S, U)
            assert np.array_equal(fmt, want), (S, trial, U, fmt, want)


def test_zero_option_equals_bruteforce_all_bands():
    rng = np.random.default_rng(77)
    tex, s1, s7, vmin, vmax = _scene(rng, 16)
    for U in (9, 17):
        fmt = O.rate_select_zero(s1, s7, O.band_hist(tex), vmin, vmax, (U + 2) / 4, 16)
        assert np.array_equal(fmt, _brute(_distortions(s1, s7, tex, vmin, vmax, 16), 16, U))


def test_zero_option_dropped_error_is_the_squared_values():
    """Brute force over distortions with the dropped band's error summed
    texel by texel picks the same bands (random data, no near-ties)."""
    rng = np.random.default_rng(5)
    for trial in range(10):
        tex, s1, s7, vmin, vmax = _scene(rng, 9)
        D = _distortions(s1, s7, tex, vmin, vmax, 9, direct=True)
        for U in (3, 8, 12):
            fmt = O.rate_select_zero(s1, s7, O.band_hist(tex), vmin, vmax, (U + 2) * 4 / 9, 9)
            assert np.array_equal(fmt, _brute(D, 9, U))


def test_zero_option_budget_and_extremes():
    rng = np.random.default_rng(8)
    tex, s1, s7, vmin, vmax = _scene(rng, 16)
    h = O.band_hist(tex)
    nblk = 1000
    prev = None
    for U in range(0, 31):
        rate = (U + 2) / 4
        fmt = O.rate_select_zero(s1, s7, h, vmin, vmax, rate, 16)
        bits = sum({7: 128, 1: 64, 3: 0}[int(f)] * nblk for f in fmt)
        assert fmt[0] == 7 and bits == rate * 16 * nblk * 16
        # more bits never raise the least distortion
        D = _distortions(s1, s7, tex, vmin, vmax, 16)
        obj = sum(D[b][PREF.index(int(fmt[b]))] for b in range(1, 16))
        assert prev is None or obj <= prev * (1 + 1e-12)
        prev = obj
    assert list(O.rate_select_zero(s1, s7, h, vmin, vmax, 0.5, 16)) == [7] + [3] * 15
    assert list(O.rate_select_zero(s1, s7, h, vmin, vmax, 8.0, 16)) == [7] * 16
    for rate in (0.25, 0.4, 8.25, 6.1, -1.0):
        assert O.rate_select_zero(s1, s7, h, vmin, vmax, rate, 16) is None
    assert list(O.rate_select_zero(s1[:1], s7[:1], h[:1], vmin, vmax, 8.0, 1)) == [7]
    assert O.rate_select_zero(s1, s7, h, vmin, vmax, 4.0, 1) is None


def test_zero_option_without_useful_drops_is_the_top_k_rule():
    """When dropping any band costs more than all else (large values), the
    choice at a budget that needs no drop is the k-largest-gain rule."""
    rng = np.random.default_rng(9)
    for S in (4, 9, 16):
        tex, s1, s7, vmin, vmax = _scene(rng, S)
        vmin = (vmin + 1000.0).astype(np.float32)
        vmax = (vmax + 1000.0).astype(np.float32)
        h = O.band_hist(tex)
        for k in range(S):
            rate = (S + 1 + k) * 4 / S
            assert np.array_equal(O.rate_select_zero(s1, s7, h, vmin, vmax, rate, S),
                                  O.rate_select(s1, s7, vmin, vmax, rate, S)), (S, k)


def test_zero_option_ties_and_zero_bands():
    """Identical bands tie: the lower band gets the larger format (BC7,
    then BC1, then none).  A band whose values are all exactly zero is
    dropped first."""
    rng = np.random.default_rng(10)
    tex, s1, s7, vmin, vmax = _scene(rng, 4)
    tex[2] = tex[1]
    s1[2], s7[2], vmin[2], vmax[2] = s1[1], s7[1], vmin[1], vmax[1]
    tex[3] = tex[1]
    s1[3], s7[3], vmin[3], vmax[3] = s1[1], s7[1], vmin[1], vmax[1]
    vmin = (vmin + 1000.0).astype(np.float32)   # dropping costs more than any coding
    vmax = (vmax + 1000.0).astype(np.float32)
    h = O.band_hist(tex)
    assert list(O.rate_select_zero(s1, s7, h, vmin, vmax, (4 + 2) * 4 / 4, 4)) == [7, 7, 1, 1]
    assert list(O.rate_select_zero(s1, s7, h, vmin, vmax, (1 + 2) * 4 / 4, 4)) == [7, 1, 3, 3]
    tex, s1, s7, vmin, vmax = _scene(rng, 9)
    tex[5] = 0
    vmin[5], vmax[5] = 0.0, 0.0
    s1[5] = s7[5] = 0
    fmt = O.rate_select_zero(s1, s7, O.band_hist(tex), vmin, vmax, (7 + 2) * 4 / 9, 9)
    assert fmt[5] == 3


def test_rate_select_class_scenes():
    """The k-largest-gain rule over S bands: k = rate*S/4 - S - 1."""
    rng = np.random.default_rng(11)
    for S in (1, 4, 9):
        tex, s1, s7, vmin, vmax = _scene(rng, S)
        for k in range(S):
            fmt = O.rate_select(s1, s7, vmin, vmax, (S + 1 + k) * 4 / S, S)
            assert fmt[0] == 7 and (fmt == 7).sum() == k + 1 and (fmt[1:] != 3).all()
        assert O.rate_select(s1, s7, vmin, vmax, (S + 1 + S) * 4 / S, S) is None


def test_encode_auto_zero_round_trip():
    nblk = 24
    rng = np.random.default_rng(12)
    tex = np.stack([smooth_blocks(nblk, 200 + b, spread=2 + 3 * b) for b in range(9)])
    vmin = np.full(16, -0.5, np.float32)
    vmax = np.full(16, 0.5, np.float32)
    rate = (9 + 2) * 4 / 9
    payload, off, fmt = O.encode_auto(tex, vmin, vmax, rate, zero=True)
    assert fmt[0] == 7 and len(fmt) == 9
    assert payload.size == sum({7: 16, 1: 8, 3: 0}[int(f)] * nblk for f in fmt)
    dec = O.decode_stream(payload, off, fmt, nblk)
    for b in range(9):
        if fmt[b] == 3:
            assert not dec[b].any()
        elif fmt[b] == 7:
            assert np.array_equal(dec[b], O.bc7_decode(O.bc7_encode(tex[b])[0]))
        else:
            assert np.array_equal(dec[b], O.bc1_decode(O.bc1_encode(tex[b])[0]))
