"""GPU: the variable number of bands (Sec. IV-B) through the C ABI -- degree
classes, the class-major sort and per-class textures bit-exact against the
oracle; each class coded, batched and decoded like a scene with fewer bands,
its dropped bands decoding as zero."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2607_14513_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


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


MIX = (0.35, 0.2, 0.15, 0.3)


@pytest.mark.parametrize("n,seed,mix,small,tau,pre", [
    (1, 1, MIX, 0.0, 0.0, False), (17, 2, MIX, 0.0, 0.0, False), (4101, 3, MIX, 0.0, 0.0, False),
    (4101, 4, MIX, 1e-4, 1e-4, False), (4101, 5, MIX, 1e-4, 0.0, False), (20_000, 6, (0.5, 0.0, 0.5, 0.0), 0.0, 0.0, False),
    (65_536, 7, MIX, 1e-4, 1e-4, True), (3000, 8, None, 0.0, 0.0, False),
    # SH rows past 256 MiB: the range pass streams them (non-temporal loads)
    (1_500_000, 13, MIX, 1e-4, 1e-4, False)])
def test_reorder_degrees_bit_exact(G, n, seed, mix, small, tau, pre):
    gsbc, ctx = G
    pos, sh = synth.make_scene(n, seed=seed, degree_mix=mix, small=small)
    mu = synth.make_opacity(n, seed=seed) if pre else None
    say("reorder degrees", n, mix, tau, pre)
    perm, counts, tex, descs = ctx.reorder_degrees(dev(pos), dev(sh), tau=tau, opacity=dev(mu) if pre else None,
                                                   params=gsbc.default_params(quantiser=int(pre)))
    rperm, rcounts, rtex, rvmin, rvmax = O.reorder_degrees(pos, sh, tau, opacity=mu, quantiser=int(pre))
    assert counts == rcounts.tolist()
    assert np.array_equal(host(perm).view(np.uint32), rperm)
    for L in range(4):
        d = descs[L]
        assert d.n_prims == counts[L] and d.n_streams == (L + 1) ** 2 and d.arrangement == gsbc.ARR_BANDS
        assert np.array_equal(d.ranges()[0].view(np.uint32), rvmin.view(np.uint32))
        assert np.array_equal(d.ranges()[1].view(np.uint32), rvmax.view(np.uint32))
        if counts[L] == 0:
            assert tex[L] is None and rtex[L] is None
        else:
            assert np.array_equal(host(tex[L]), rtex[L]), L
    if mix is None:                       # nothing dropped: class 3 is the plain reorder
        assert counts == [0, 0, 0, n]
        p2, t2, _ = ctx.reorder(dev(pos), dev(sh))
        assert np.array_equal(host(p2), host(perm)) and np.array_equal(host(t2), host(tex[3]))


def test_classes_encode_batch_and_decode(G):
    gsbc, ctx = G
    n = 20_011
    pos, sh = synth.make_scene(n, seed=9, degree_mix=MIX)
    perm, counts, tex, descs = ctx.reorder_degrees(dev(pos), dev(sh))
    rperm, rcounts, rtex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0)
    start = np.concatenate([[0], np.cumsum(counts)])
    dirs = synth.make_dirs(12, seed=9)
    texs, dl, ref = [], [], []
    for L in range(4):
        if counts[L] == 0:
            continue
        nb = (L + 1) ** 2
        fmt = np.array([7] + [1] * (nb - 1), np.uint8)
        d = descs[L]
        for k, f in enumerate(fmt):
            d.format[k] = int(f)
        say("class", L, counts[L])
        blocks, d2, sse = ctx.encode(tex[L], d, fmt=gsbc.FMT_BANDS, want_sse=True)
        rpay, roff, rsse = O.encode(rtex[L], fmt)
        assert np.array_equal(host(blocks)[:rpay.size], rpay)
        assert np.array_equal(d2.offsets(), roff)
        assert np.array_equal(np.where(fmt == 1, sse[0][:nb], sse[1][:nb]), rsse)
        assert np.array_equal(host(ctx.decode(blocks, d2)), O.decode_stream(rpay, roff, fmt, rtex[L].shape[1]))
        # colours of the class: dropped bands contribute nothing
        out = host(ctx.decode_eval(blocks, d2, dev(dirs)))
        slots = np.arange(counts[L], dtype=np.uint32)
        r, sc = O.decode_eval(rpay, roff, fmt, vmin, vmax, dirs, slots)
        err = np.abs(out.astype(np.float64) - r)
        assert np.all(err <= REL_TOL * sc), (L, float((err / np.maximum(sc, 1e-30)).max()))
        part = perm[start[L]:start[L + 1]].contiguous()
        view = np.array([0.2, 1.7, -0.4], np.float32)
        ov = host(ctx.decode_eval_view(blocks, d2, dev(pos), part, view))
        rv, sv = O.decode_eval_view(rpay, roff, fmt, vmin, vmax, pos, rperm[start[L]:start[L + 1]], view, slots)
        err = np.abs(ov.astype(np.float64) - rv)
        assert np.all(err <= REL_TOL * sv), L
        # the rate controller over the class's bands (exact budget, as the oracle)
        for mode, rate in ((gsbc.FMT_AUTO, (nb + 1 + nb // 2) * 4 / nb), (gsbc.FMT_AUTO_ZERO, (nb // 2 + 2) * 4 / nb)):
            ab, ad, _ = ctx.encode(tex[L], d, fmt=mode, rate=rate)
            apay, aoff, afmt = O.encode_auto(rtex[L], vmin, vmax, rate, zero=mode == gsbc.FMT_AUTO_ZERO)
            assert np.array_equal(ad.formats(), afmt) and np.array_equal(ad.offsets(), aoff), (L, mode)
            assert ad.payload_bytes == apay.size and np.array_equal(host(ab)[:apay.size], apay), (L, mode)
        texs.append(tex[L])
        dl.append(d)
        ref.append((rpay, d2))
    blocks = [torch.zeros(r[1].payload_bytes + 64, dtype=torch.uint8, device="cuda") for r in ref]
    outd, _ = ctx.encode_batch(texs, dl, blocks)
    for i, (rpay, d2) in enumerate(ref):
        assert np.array_equal(host(blocks[i])[:rpay.size], rpay), i


def test_degrees_full_size_sampled(G):
    """The degree-class workload at the size the bench times it: 1,048,576
    primitives (32 clusters, 64-component DC mixture) whose SH degrees are
    drawn as 35/20/15/30 %.  Class counts, the class-major permutation, the
    ranges and every class's textures bit-exact against the oracle; the
    classes coded band 0 BC7 + the rest BC1 in one batch equal the same
    classes coded one by one, and 256 blocks of every kept band of every
    class (first and last included) equal the oracle's encoder."""
    gsbc, ctx = G
    c = synth.CONFIGS["mid"]
    pos, sh = synth.make_scene(c["n"], c["clusters"], c["comps"], c["seed"] + 100, degree_mix=MIX)
    say("degrees full size: reorder")
    perm, counts, tex, descs = ctx.reorder_degrees(dev(pos), dev(sh))
    rperm, rcounts, rtex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0)
    assert counts == rcounts.tolist() and all(counts)
    assert np.array_equal(host(perm).view(np.uint32), rperm)
    texs, dl, single = [], [], []
    for L in range(4):
        nb = (L + 1) ** 2
        d = descs[L]
        assert np.array_equal(d.ranges()[0].view(np.uint32), vmin.view(np.uint32))
        assert np.array_equal(d.ranges()[1].view(np.uint32), vmax.view(np.uint32))
        assert np.array_equal(host(tex[L]), rtex[L]), L
        fmt = [7] + [1] * (nb - 1)
        for k, f in enumerate(fmt):
            d.format[k] = f
        say("degrees full size: class", L, counts[L])
        blocks, d2, _ = ctx.encode(tex[L], d, fmt=gsbc.FMT_BANDS)
        hb = host(blocks)
        nblk = d2.blocks_per_stream
        for k, f in enumerate(fmt):
            pick = _sample_blocks(nblk, 256, 40 * L + k)
            bs = 16 if f == 7 else 8
            stream = hb[int(d2.offsets()[k]):int(d2.offsets()[k]) + nblk * bs].reshape(nblk, bs)
            ref = O.bc7_encode(rtex[L][k][pick])[0] if f == 7 else O.bc1_encode(rtex[L][k][pick])[0]
            assert np.array_equal(stream[pick], ref), (L, k)
        texs.append(tex[L])
        dl.append(d)
        single.append(hb[:d2.payload_bytes])
    say("degrees full size: batch")
    outs = [torch.zeros(p.size + 64, dtype=torch.uint8, device="cuda") for p in single]
    ctx.encode_batch(texs, dl, outs)
    for L, p in enumerate(single):
        assert np.array_equal(host(outs[L])[:p.size], p), L


def _sample_blocks(nblk, count, seed):
    """count distinct block indices of a stream, its first and last included."""
    rng = np.random.default_rng(seed)
    inner = 1 + rng.choice(max(nblk - 2, 0), min(max(nblk - 2, 0), count - 2), replace=False)
    return np.unique(np.concatenate([[0, nblk - 1], inner]))


def test_degree_errors(G):
    gsbc, ctx = G
    pos, sh = synth.make_scene(100, seed=10)
    for kw in ({"tau": -1.0}, {"tau": float("nan")}, {"params": gsbc.default_params(order=1)},
               {"params": gsbc.default_params(arrangement=1)}):
        with pytest.raises(gsbc.GsbcError) as e:
            ctx.reorder_degrees(dev(pos), dev(sh), **kw)
        assert e.value.status == gsbc.E_ARG, kw


@pytest.mark.parametrize("n,seed,mix,tau", [(1, 11, (0.0, 1.0, 0.0, 0.0), 0.0), (19, 12, MIX, 0.0),
                                            (4101, 13, MIX, 1e-4), (65_536, 14, MIX, 0.0)])
def test_setup_c_class_bit_exact(G, n, seed, mix, tau):
    """Fig. SetupC for the degree-1 class: permutation, counts and every
    class texture bit-exact against the oracle; the class is one stream of
    pad16/4 blocks, the other classes unchanged."""
    gsbc, ctx = G
    pos, sh = synth.make_scene(n, seed=seed, degree_mix=mix, small=1e-4 if tau else 0.0)
    say("reorder degrees SetupC", n, mix, tau)
    perm, counts, tex, descs = ctx.reorder_degrees(dev(pos), dev(sh), tau=tau,
                                                   params=gsbc.default_params(arrangement=gsbc.ARR_QUAD))
    rperm, rcounts, rtex, _, _ = O.reorder_degrees(pos, sh, tau, arrangement=O.ARR_QUAD)
    assert counts == rcounts.tolist()
    assert np.array_equal(host(perm).view(np.uint32), rperm)
    for L in range(4):
        d = descs[L]
        if L == 1:
            assert d.arrangement == gsbc.ARR_QUAD and d.n_streams == 1 and d.blocks_per_stream == d.n_pad // 4
        else:
            assert d.arrangement == gsbc.ARR_BANDS and d.n_streams == (L + 1) ** 2
        if counts[L] == 0:
            assert tex[L] is None and rtex[L] is None
        else:
            assert np.array_equal(host(tex[L]), rtex[L]), L


def test_setup_c_encode_decode_and_container(G, tmp_path):
    """The Fig. SetupC class coded in BC1 and in BC7, alone and in a batch,
    decoded whole, by direction and by view position, and through a
    container file: bitstreams and texels bit-exact, colours within 1e-5 of
    the FP64 oracle."""
    gsbc, ctx = G
    n = 20_011
    pos, sh = synth.make_scene(n, seed=15, degree_mix=MIX)
    perm, counts, tex, descs = ctx.reorder_degrees(dev(pos), dev(sh),
                                                   params=gsbc.default_params(arrangement=gsbc.ARR_QUAD))
    rperm, rcounts, rtex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0, arrangement=O.ARR_QUAD)
    c1 = counts[1]
    s1 = counts[0]
    slots = np.arange(c1, dtype=np.uint32)
    dirs = synth.make_dirs(9, seed=15)
    view = np.array([-0.3, 1.1, 0.6], np.float32)
    for f in (1, 7):
        d = descs[1]
        d.format[0] = f
        fmt = np.array([f], np.uint8)
        say("SetupC class", c1, "format", f)
        blocks, d2, _ = ctx.encode(tex[1], d, fmt=gsbc.FMT_BANDS)
        rpay, roff, _ = O.encode(rtex[1], fmt)
        assert np.array_equal(host(blocks)[:rpay.size], rpay) and d2.payload_bytes == rpay.size
        assert np.array_equal(host(ctx.decode(blocks, d2)), O.decode_stream(rpay, roff, fmt, rtex[1].shape[1]))
        out = host(ctx.decode_eval(blocks, d2, dev(dirs)))
        r, sc = O.decode_eval(rpay, roff, fmt, vmin, vmax, dirs, slots, arrangement=O.ARR_QUAD)
        bad = np.argwhere(np.abs(out.astype(np.float64) - r) > REL_TOL * sc)
        assert bad.size == 0, (f, len(bad), bad[:8].tolist(), [(float(out[tuple(i)]), float(r[tuple(i)]))
                                                                 for i in bad[:4]])
        part = perm[s1:s1 + c1].contiguous()
        ov = host(ctx.decode_eval_view(blocks, d2, dev(pos), part, view))
        rv, sv = O.decode_eval_view(rpay, roff, fmt, vmin, vmax, pos, rperm[s1:s1 + c1], view, slots,
                                    arrangement=O.ARR_QUAD)
        assert np.all(np.abs(ov.astype(np.float64) - rv) <= REL_TOL * sv), f
        path = str(tmp_path / f"setup_c_{f}.gsbc")
        ctx.save(path, blocks, d2)
        b3, d3 = ctx.load(path)
        assert d3.arrangement == gsbc.ARR_QUAD and d3.n_streams == 1
        assert np.array_equal(host(b3)[:rpay.size], rpay)
        assert np.array_equal(host(ctx.decode_eval(b3, d3, dev(dirs))), out)
        with pytest.raises(gsbc.GsbcError) as e:
            ctx.encode(tex[1], d, fmt=gsbc.FMT_AUTO, rate=6.0)
        assert e.value.status == gsbc.E_UNSUPPORTED
    # the class in a batch beside a per-band class
    d1 = descs[1]
    d1.format[0] = 7
    d3 = descs[3]
    for k in range(16):
        d3.format[k] = 7 if k == 0 else 1
    ref = [O.encode(rtex[1], np.array([7], np.uint8))[0],
           O.encode(rtex[3], np.array([7] + [1] * 15, np.uint8))[0]]
    outb = [torch.zeros(r.size + 64, dtype=torch.uint8, device="cuda") for r in ref]
    ctx.encode_batch([tex[1], tex[3]], [d1, d3], outb)
    for i, r in enumerate(ref):
        assert np.array_equal(host(outb[i])[:r.size], r), i
