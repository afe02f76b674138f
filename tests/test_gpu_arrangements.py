"""GPU: the block arrangements of Sec. IV-B through the C ABI -- Fig. SetupA
(one primitive per block, one stream) and Fig. SetupB (four primitives per
four blocks, four streams) -- against the oracle: textures, bitstreams and
SSEs bit-exact, decoded textures bit-exact, colours within the FP64 bound;
the container and the batched encoder carry the arrangement."""
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


ARRS = [(1, "prim"), (2, "quad")]


@pytest.mark.parametrize("arr", [1, 2])
@pytest.mark.parametrize("n,seed,order,pre", [(1, 81, 0, False), (17, 82, 0, False), (4101, 83, 0, True),
                                              (4101, 84, 1, False), (65_536, 85, 0, False)])
def test_reorder_arrangement_bit_exact(G, arr, n, seed, order, pre):
    gsbc, ctx = G
    pos, sh = synth.make_scene(n, seed=seed)
    mu = synth.make_opacity(n, seed=seed) if pre else None
    say("reorder arrangement", arr, n, order, pre)
    params = gsbc.default_params(arrangement=arr, order=order, quantiser=int(pre))
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), params=params, opacity=dev(mu) if pre else None)
    if order == 0:
        rperm, rtex, rvmin, rvmax = O.reorder(pos, sh, opacity=mu, quantiser=int(pre), arrangement=arr)
    else:
        rvmin, rvmax = O.band_range(sh)
        rperm = np.arange(n, dtype=np.uint32)
        rtex = O.pack(O.quantise(sh, rvmin, rvmax), rperm, arr)
    assert (d.arrangement, d.n_streams) == (arr, O.N_STREAMS[arr])
    assert d.blocks_per_stream * d.n_streams == d.n_pad
    assert np.array_equal(host(perm).view(np.uint32), rperm)
    assert tex.shape == rtex.shape
    assert np.array_equal(host(tex), rtex)
    assert np.array_equal(d.ranges()[0].view(np.uint32), rvmin.view(np.uint32))


FMTS = {1: [[7], [1]], 2: [[7, 1, 1, 1], [1, 7, 7, 1], [1, 1, 1, 1]]}


@pytest.mark.parametrize("arr,which", [(1, 0), (1, 1), (2, 0), (2, 1), (2, 2)])
@pytest.mark.parametrize("n", [4101, 65_536])
def test_encode_arrangement_bit_exact(G, arr, which, n):
    gsbc, ctx = G
    fmt = np.array(FMTS[arr][which], np.uint8)
    pos, sh = synth.make_scene(n, seed=90 + arr)
    _, tex, d = ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=arr))
    for k, f in enumerate(fmt):
        d.format[k] = int(f)
    say("encode arrangement", arr, fmt.tolist(), n)
    blocks, d2, sse = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS, want_sse=True)
    _, rtex, _, _ = O.reorder(pos, sh, arrangement=arr)
    rpay, roff, rsse = O.encode(rtex, fmt)
    assert np.array_equal(d2.formats(), fmt)
    assert np.array_equal(d2.offsets(), roff)
    assert d2.payload_bytes == rpay.size
    assert np.array_equal(host(blocks)[:rpay.size], rpay)
    got = np.where(fmt == 1, sse[0][:len(fmt)], sse[1][:len(fmt)])
    assert np.array_equal(got, rsse)
    assert np.all(sse[:, len(fmt):] == -1)
    # decoded textures
    assert np.array_equal(host(ctx.decode(blocks, d2)), O.decode_stream(rpay, roff, fmt, rtex.shape[1]))


@pytest.mark.parametrize("arr,order", [(1, 0), (2, 0), (2, 1)])
def test_arrangement_full_size_sampled(G, arr, order):
    """At the size the bench codes the arrangements (1,048,576 primitives, 32
    clusters, 64-component DC mixture; sorted and input order): permutation
    and every stream's texture bit-exact against the oracle's packer, then
    the first format set coded and 256 blocks of every stream (first and
    last included) equal to the oracle's encoder."""
    gsbc, ctx = G
    c = synth.CONFIGS["mid"]
    pos, sh = synth.make_scene(c["n"], c["clusters"], c["comps"], c["seed"])
    say("arrangement full size", arr, order)
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=arr, order=order))
    if order == 0:
        rperm, rtex, _, _ = O.reorder(pos, sh, arrangement=arr)
    else:
        rvmin, rvmax = O.band_range(sh)
        rperm = np.arange(c["n"], dtype=np.uint32)
        rtex = O.pack(O.quantise(sh, rvmin, rvmax), rperm, arr)
    assert np.array_equal(host(perm).view(np.uint32), rperm)
    assert np.array_equal(host(tex), rtex)
    fmt = np.array(FMTS[arr][0], np.uint8)
    for k, f in enumerate(fmt):
        d.format[k] = int(f)
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS)
    hb = host(blocks)
    nblk = d2.blocks_per_stream
    for k, f in enumerate(fmt):
        rng = np.random.default_rng(70 + 8 * arr + k)
        pick = np.unique(np.concatenate([[0, nblk - 1], rng.choice(nblk, 254, replace=False)]))
        bs = 16 if f == 7 else 8
        stream = hb[int(d2.offsets()[k]):int(d2.offsets()[k]) + nblk * bs].reshape(nblk, bs)
        ref = O.bc7_encode(rtex[k][pick])[0] if f == 7 else O.bc1_encode(rtex[k][pick])[0]
        assert np.array_equal(stream[pick], ref), (arr, k)


@pytest.mark.parametrize("arr", [1, 2])
def test_whole_format_and_auto(G, arr):
    gsbc, ctx = G
    n = 2000 + 7
    pos, sh = synth.make_scene(n, seed=95)
    _, tex, d = ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=arr))
    _, rtex, _, _ = O.reorder(pos, sh, arrangement=arr)
    S = O.N_STREAMS[arr]
    for f in (gsbc.FMT_BC1, gsbc.FMT_BC7):
        blocks, d2, _ = ctx.encode(tex, d, fmt=f)
        rpay, _, _ = O.encode(rtex, np.full(S, f, np.uint8))
        assert np.array_equal(host(blocks)[:rpay.size], rpay)
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode(tex, d, fmt=gsbc.FMT_AUTO, rate=6.0)
    assert e.value.status == gsbc.E_UNSUPPORTED
    bad = d.copy()
    bad.n_streams = 16
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode(tex, bad, fmt=gsbc.FMT_BC1)
    assert e.value.status == gsbc.E_ARG
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=3))
    assert e.value.status == gsbc.E_ARG


@pytest.mark.parametrize("arr", [1, 2])
@pytest.mark.parametrize("n,V", [(4101, 40), (65_536, 8)])
def test_decode_eval_arrangement(G, arr, n, V):
    gsbc, ctx = G
    fmt = np.array(FMTS[arr][0], np.uint8)
    pos, sh = synth.make_scene(n, seed=97)
    perm, tex, d = ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=arr))
    for k, f in enumerate(fmt):
        d.format[k] = int(f)
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS)
    _, rtex, vmin, vmax = O.reorder(pos, sh, arrangement=arr)
    rpay, roff, _ = O.encode(rtex, fmt)
    assert np.array_equal(host(blocks)[:rpay.size], rpay)
    dirs = synth.make_dirs(V, seed=97)
    say("decode_eval arrangement", arr, n, V)
    out = host(ctx.decode_eval(blocks, d2, dev(dirs)))
    slots = np.arange(n, dtype=np.uint32)
    ref, scale = O.decode_eval(rpay, roff, fmt, vmin, vmax, dirs, slots, arrangement=arr)
    err = np.abs(out.astype(np.float64) - ref)
    assert np.all(err <= REL_TOL * scale), float((err / np.maximum(scale, 1e-30)).max())
    view = np.array([0.5, 0.5, 2.5], np.float32)
    ov = host(ctx.decode_eval_view(blocks, d2, dev(pos), perm, view))
    rv, sv = O.decode_eval_view(rpay, roff, fmt, vmin, vmax, pos, host(perm).view(np.uint32), view, slots,
                                arrangement=arr)
    err = np.abs(ov.astype(np.float64) - rv)
    assert np.all(err <= REL_TOL * sv), float((err / np.maximum(sv, 1e-30)).max())


def test_container_and_batch_carry_the_arrangement(G, tmp_path):
    gsbc, ctx = G
    scenes = []
    for i, (arr, n) in enumerate([(2, 333), (0, 4101), (1, 1000 + 1), (2, 20_000)]):
        pos, sh = synth.make_scene(n, seed=100 + i)
        _, tex, d = ctx.reorder(dev(pos), dev(sh), params=gsbc.default_params(arrangement=arr))
        fmt = [7] + [1] * (d.n_streams - 1) if d.n_streams > 1 else [7]
        for k, f in enumerate(fmt):
            d.format[k] = f
        scenes.append((tex, d))
    ref = []
    for tex, d in scenes:
        b, d2, sse = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS, want_sse=True)
        ref.append((host(b)[:d2.payload_bytes], d2, sse))
    blocks = [torch.zeros(r[1].payload_bytes + 64, dtype=torch.uint8, device="cuda") for r in ref]
    outd, sse = ctx.encode_batch([s[0] for s in scenes], [s[1] for s in scenes], blocks, want_sse=True)
    for i, (rpay, rd, rsse) in enumerate(ref):
        assert np.array_equal(host(blocks[i])[:rd.payload_bytes], rpay), i
        assert np.array_equal(outd[i].offsets(), rd.offsets())
        f = rd.formats()
        assert np.array_equal(sse[i][:len(f)], np.where(f == 1, rsse[0][:len(f)], rsse[1][:len(f)]))
    # container round trip of the SetupB scene
    path = str(tmp_path / "quad.gsbc")
    b0 = dev(ref[0][0])
    ctx.save(path, b0, ref[0][1])
    b2, d3 = ctx.load(path)
    assert bytes(d3) == bytes(ref[0][1])
    assert (d3.arrangement, d3.n_streams) == (2, 4)
    dirs = dev(synth.make_dirs(3, seed=1))
    assert np.array_equal(host(ctx.decode_eval(b2, d3, dirs)), host(ctx.decode_eval(b0, ref[0][1], dirs)))
