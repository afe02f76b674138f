"""GPU: the colour stage of a tile rasteriser (Sec. II, eqs. blend,
preblend, premult) through the C ABI against the oracle's FP64 blend.

Bound (FP32 against FP64, per pixel and channel, for a list of L entries):
  |a32 - a64| <= 3e-5 * sum_i g_i T_i |c~_i| + 4 * 2^-24 * sum_i i g_i |c~_i|
                 + (L + 1) * 2^-120
where |c~_i| = sum_k |Htilde_ik Y_k|.  The first term covers each colour's
FP32 evaluation (within 1e-5 of its term size, the view decode's bound) and
the FP32 footprint g (q and exp, within 2e-5 where g matters); the second
the transmittance, whose i-th factor product carries an absolute error of at
most about 3 i roundings of 2^-24 (each factor 1 - mu g <= 1); the third
FP32 underflow (g T below 2^-126 flushed, times colours well under 64).
The final transmittance is checked against 3 (L + 1) 2^-24."""
import sys

import numpy as np
import pytest

import oracle as O
from conftest import oracle_blend_tiles_subset
from paper_2607_14513_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -24
VIEW = np.array([0.5, 0.45, 2.5], np.float32)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2607_14513_amd import gsbc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = gsbc.Context(0)
    yield gsbc, ctx
    ctx.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _check(img, T, ref, ts, tx, ty):
    r, rt, b, bt = ref
    L = np.diff(ts.astype(np.int64)).reshape(ty, tx)
    Lpix = np.repeat(np.repeat(L, 16, 0), 16, 1)
    err = np.abs(img.astype(np.float64) - r)
    lim = 3e-5 * b + 4 * U * bt + (Lpix[..., None] + 1) * 2.0 ** -120
    assert np.all(err <= lim), float((err - lim).max())
    assert np.all(np.abs(T.astype(np.float64) - rt) <= 3 * (Lpix + 1) * U)


@pytest.mark.parametrize("n,tiles,seed,fmt", [
    (3000, (8, 6), 3, [7] + [1] * 15),
    (20_011, (20, 15), 4, [7, 7, 1, 3, 1, 7, 3, 1, 1, 3, 1, 1, 3, 1, 3, 3]),
    (600, (3, 2), 5, [7] * 16)])
def test_blend_tiles_matches_oracle(G, n, tiles, seed, fmt):
    gsbc, ctx = G
    tx, ty = tiles
    pos, sh = synth.make_scene(n, seed=seed)
    mu = synth.make_opacity(n, seed=seed)
    fmt = np.array(fmt, np.uint8)
    rperm, rtex, vmin, vmax = O.reorder(pos, sh, opacity=mu)
    rpay, roff, _ = O.encode(rtex, fmt)
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), opacity=dev(mu))
    for k in range(16):
        d.format[k] = int(fmt[k])
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS)
    foot, ts, lst = synth.make_tiles(pos, VIEW, tx, ty, seed=seed)
    say("blend", n, tiles, int(ts[-1]), "entries")
    gslot = np.argsort(host(perm).view(np.uint32)).astype(np.int32)
    rslot = np.argsort(rperm).astype(np.uint32)
    img, T = ctx.blend_tiles(blocks, d2, dev(pos), perm, VIEW, dev(mu), dev(foot), dev(ts.astype(np.int32)),
                             dev(gslot[lst]), tx, ty)
    ref = O.blend_tiles(rpay, roff, fmt, vmin, vmax, pos, rperm, VIEW, mu, foot, ts, rslot[lst], tx, ty)
    _check(host(img), host(T), ref, ts, tx, ty)
    assert np.diff(ts.astype(np.int64)).max() > 256          # several LDS chunks per tile


def test_blend_tiles_edges(G):
    """Empty tiles, single entries, an id past the scene (NaN), tile bounds
    past the list's end (clamped), no transmittance output."""
    gsbc, ctx = G
    n = 700
    pos, sh = synth.make_scene(n, seed=6)
    mu = synth.make_opacity(n, seed=6)
    fmt = np.array([7] + [1] * 15, np.uint8)
    rperm, rtex, vmin, vmax = O.reorder(pos, sh, opacity=mu)
    rpay, roff, _ = O.encode(rtex, fmt)
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), opacity=dev(mu))
    for k in range(16):
        d.format[k] = int(fmt[k])
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS)
    foot, _, _ = synth.make_tiles(pos, VIEW, 2, 2, seed=6)
    lst = np.array([5, 9, 9, 600, 2, 77, 13], np.uint32)      # slot ids
    ts = np.array([0, 0, 1, 4, 30], np.uint32)               # tile 3 runs past the list: clamped to 7
    img, T = ctx.blend_tiles(blocks, d2, dev(pos), perm, VIEW, dev(mu), dev(foot), dev(ts.astype(np.int32)),
                             dev(lst.astype(np.int32)), 2, 2)
    img = host(img)
    ts_c = np.minimum(ts, lst.size)
    ref = O.blend_tiles(rpay, roff, fmt, vmin, vmax, pos, rperm, VIEW, mu, foot, ts_c, lst, 2, 2)
    _check(img, host(T), ref, ts_c, 2, 2)
    assert not img[:16, :16].any() and (host(T)[:16, :16] == 1.0).all()
    bad = lst.copy()
    bad[1] = n + 5
    img2, T2 = ctx.blend_tiles(blocks, d2, dev(pos), perm, VIEW, dev(mu), dev(foot), dev(ts.astype(np.int32)),
                               dev(bad.astype(np.int32)), 2, 2, want_transmittance=False)
    img2 = host(img2)
    # entry 1 belongs to tile 2 (tx 0, ty 1): that tile is NaN, the others unchanged
    assert T2 is None and np.isnan(img2[16:, :16]).all()
    assert np.array_equal(img2[:, 16:], img[:, 16:]) and np.array_equal(img2[:16, :16], img[:16, :16])
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.blend_tiles(blocks, d2, dev(pos), perm, (0.0, float("inf"), 0.0), dev(mu), dev(foot),
                        dev(ts.astype(np.int32)), dev(lst.astype(np.int32)), 2, 2)
    assert e.value.status == gsbc.E_ARG


@pytest.mark.parametrize("n,tiles,seed", [(3000, (8, 6), 3), (20_011, (20, 15), 4)])
def test_blend_tiles_colours_equals_fused(G, n, tiles, seed):
    """The two-pass form (view decode of every slot, then the blend reading
    those colours) gives the fused stage's image and transmittance bit for
    bit, and so the same oracle bound; ids past the scene still give NaN."""
    gsbc, ctx = G
    tx, ty = tiles
    pos, sh = synth.make_scene(n, seed=seed)
    mu = synth.make_opacity(n, seed=seed)
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), opacity=dev(mu))
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_AUTO, rate=6.0)
    foot, ts, lst = synth.make_tiles(pos, VIEW, tx, ty, seed=seed)
    gslot = np.argsort(host(perm).view(np.uint32)).astype(np.int32)
    say("blend two-pass", n, tiles, int(ts[-1]), "entries")
    pd, md, fd, tsd, ld = dev(pos), dev(mu), dev(foot), dev(ts.astype(np.int32)), dev(gslot[lst])
    img, T = ctx.blend_tiles(blocks, d2, pd, perm, VIEW, md, fd, tsd, ld, tx, ty)
    cols = ctx.decode_eval_view(blocks, d2, pd, perm, VIEW)
    img2, T2 = ctx.blend_tiles_colours(cols, perm, md, fd, tsd, ld, tx, ty)
    assert np.array_equal(host(img).view(np.uint32), host(img2).view(np.uint32))
    assert np.array_equal(host(T).view(np.uint32), host(T2).view(np.uint32))
    bad = gslot[lst].copy()
    bad[0] = n + 3                                            # first entry of the first non-empty tile
    img3, _ = ctx.blend_tiles_colours(cols, perm, md, fd, tsd, dev(bad), tx, ty, want_transmittance=False)
    img3 = host(img3)
    t0 = int(np.searchsorted(ts, 0, side="right")) - 1        # the tile holding entry 0
    yy, xx = divmod(t0, tx)
    assert np.isnan(img3[16 * yy:16 * yy + 16, 16 * xx:16 * xx + 16]).all()
    with pytest.raises(ValueError):
        ctx.blend_tiles_colours(cols[:, :2].contiguous(), perm, md, fd, tsd, ld, tx, ty)


def test_blend_tiles_full_size_sampled(G):
    """The colour stage at the size the bench times it: the 3,145,728-
    primitive scene (256 clusters), a 1920 x 1088 image of 120 x 68 tiles
    whose lists come from projecting the scene from one view position
    (footprint sigmas 0.7-6 px, 16.6 M entries), 6 bits/texel (band 0 and
    seven other bands BC7, the rest BC1).  The fused and two-pass forms give
    the same bits over the whole image; seven tiles (lists of 300 to 8,000
    entries, several LDS chunks each, plus one short list) against the FP64
    oracle on oracle-encoded blocks, the other tiles' lists left empty on
    the oracle side."""
    gsbc, ctx = G
    c = synth.CONFIGS["large"]
    n, tx, ty = c["n"], 120, 68
    view = np.array([0.5, 0.5, 2.5], np.float32)
    pos, sh = synth.make_scene(n, c["clusters"], c["comps"], c["seed"])
    mu = synth.make_opacity(n, seed=c["seed"])
    fmt = np.array([7, 7, 1, 7, 1, 7, 1, 7, 1, 7, 1, 7, 1, 1, 7, 1], np.uint8)
    assert 8 * (fmt == 7).sum() + 4 * (fmt == 1).sum() == 6 * 16
    say("blend full size: reorder + encode")
    perm, tex, d = ctx.reorder(dev(pos), dev(sh))
    for k in range(16):
        d.format[k] = int(fmt[k])
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS)
    del tex
    foot, ts, lst = synth.make_tiles(pos, view, tx, ty, seed=c["seed"], sigma=(0.7, 6.0))
    gperm = host(perm).view(np.uint32)
    gslot = np.argsort(gperm).astype(np.int32)
    pd, md, fd, tsd, ld = dev(pos), dev(mu), dev(foot), dev(ts.astype(np.int32)), dev(gslot[lst])
    say("blend full size:", int(ts[-1]), "entries")
    img, T = ctx.blend_tiles(blocks, d2, pd, perm, view, md, fd, tsd, ld, tx, ty)
    cols = ctx.decode_eval_view(blocks, d2, pd, perm, view)
    img2, T2 = ctx.blend_tiles_colours(cols, perm, md, fd, tsd, ld, tx, ty)
    img, T = host(img), host(T)
    assert np.array_equal(img.view(np.uint32), host(img2).view(np.uint32))
    assert np.array_equal(T.view(np.uint32), host(T2).view(np.uint32))
    del img2, T2, cols
    assert np.isfinite(img).all() and ((T >= 0) & (T <= 1)).all()

    rperm, rtex, vmin, vmax = O.reorder(pos, sh)
    assert np.array_equal(gperm, rperm)
    assert np.array_equal(d2.ranges()[0].view(np.uint32), vmin.view(np.uint32))
    L = np.diff(ts.astype(np.int64))
    rng = np.random.default_rng(11)
    pick = list(rng.choice(np.flatnonzero((L >= 300) & (L <= 2500)), 5, replace=False))
    pick.append(int(rng.choice(np.flatnonzero((L >= 6000) & (L <= 8000)))))
    pick.append(int(rng.choice(np.flatnonzero((L >= 1) & (L < 256)))))
    pick = np.unique(pick)
    say("blend full size: oracle on tiles", pick.tolist())
    (r, rt, b, bt), nblk = oracle_blend_tiles_subset(rtex, fmt, vmin, vmax, pos, rperm, view, mu, foot, ts, lst, pick,
                                                     tx, ty)
    say("blend full size: oracle encoded", nblk, "blocks per band")
    for t in pick:
        yy, xx = divmod(int(t), tx)
        sl = (slice(16 * yy, 16 * yy + 16), slice(16 * xx, 16 * xx + 16))
        err = np.abs(img[sl].astype(np.float64) - r[sl])
        lim = 3e-5 * b[sl] + 4 * U * bt[sl] + (L[t] + 1) * 2.0 ** -120
        assert np.all(err <= lim), (int(t), int(L[t]), float((err - lim).max()))
        assert np.all(np.abs(T[sl].astype(np.float64) - rt[sl]) <= 3 * (L[t] + 1) * U), int(t)
