"""GPU: per-band formats and the batched encoder, through the C ABI.

Per-band formats (band 0 BC7, the rest BC1 in the paper's Sec. V scheme, and
mixed patterns) must match the oracle bit for bit.  The batched encoder codes
many scenes of uneven size in one captured launch sequence; every scene's
bitstream and band SSEs must equal the single-scene call, for every work
split, and for replays of the captured graph.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2607_14513_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _fmt_pattern(seed):
    rng = np.random.default_rng(seed)
    f = np.where(rng.random(16) < 0.4, 7, 1).astype(np.uint8)
    f[0] = 7
    return f


# scene sizes: a single primitive, ragged, several workgroup rounds, and one
# larger than a run-alignment span in every band
SCENES = [(1, 41), (333, 42), (4101, 43), (20_007, 44), (65_536, 45)]


@pytest.fixture(scope="module")
def scenes(G):
    gsbc, ctx = G
    out = []
    for i, (n, seed) in enumerate(SCENES):
        pos, sh = synth.make_scene(n, seed=seed)
        perm, tex, d = ctx.reorder(dev(pos), dev(sh))
        fmt = _fmt_pattern(100 + i) if i % 2 else np.array([7] + [1] * 15, np.uint8)
        for k in range(16):
            d.format[k] = int(fmt[k])
        out.append((pos, sh, tex, d, fmt))
    torch.cuda.synchronize()
    return out


def _plain(gsbc, ctx, tex, d):
    blocks, d2, sse = ctx.encode(tex, d, fmt=gsbc.FMT_BANDS, want_sse=True)
    fmt = d2.formats()
    band = np.where(fmt == 1, sse[0], sse[1])
    return host(blocks)[:d2.payload_bytes], d2, band


@pytest.mark.parametrize("which", [0, 1, 2])
def test_bands_format_bit_exact(G, scenes, which):
    gsbc, ctx = G
    pos, sh, tex, d, fmt = scenes[which]
    say("bands", SCENES[which], fmt.tolist())
    payload, d2, sse = _plain(gsbc, ctx, tex, d)
    _, rtex, _, _ = O.reorder(pos, sh)
    rpay, roff, rsse = O.encode(rtex, fmt)
    assert np.array_equal(d2.offsets(), roff)
    assert d2.payload_bytes == rpay.size
    assert np.array_equal(payload, rpay)
    assert np.array_equal(sse, rsse)


TUNINGS = [
    {},
    {"item_rounds": 3, "wgs_per_cu": 2, "bc1_lanes": 64, "bc7_split": 1, "concurrent": 1},
    {"item_rounds": 1, "wgs_per_cu": 1, "bc1_lanes": 256, "bc7_split": 2, "concurrent": 0},
    {"item_rounds": 8, "wgs_per_cu": 4, "bc1_lanes": 128, "bc7_split": 0, "concurrent": 1},
    {"item_rounds": 2, "wgs_per_cu": 0, "bc1_lanes": 128, "bc7_split": 3, "concurrent": 1},
    {"item_rounds": 1, "wgs_per_cu": 3, "bc1_lanes": 64, "bc7_split": 3, "concurrent": 0},
]


@pytest.mark.parametrize("tune", range(len(TUNINGS)))
def test_batch_equals_plain(G, scenes, tune):
    gsbc, ctx = G
    t = gsbc.default_batch_tuning(**TUNINGS[tune])
    say("batch", t.as_dict())
    ref = [_plain(gsbc, ctx, tex, d) for (_, _, tex, d, _) in scenes]
    texs = [s[2] for s in scenes]
    descs = [s[3] for s in scenes]
    blocks = [torch.full((r[1].payload_bytes + 64,), 0xAB, dtype=torch.uint8, device="cuda") for r in ref]
    for call in range(2):            # the second call replays the captured graph
        for b in blocks:
            b.fill_(0xAB)
        outd, sse = ctx.encode_batch(texs, descs, blocks, tuning=t, want_sse=True)
        for i, (rpay, rd, rsse) in enumerate(ref):
            assert np.array_equal(outd[i].offsets(), rd.offsets()), (call, i)
            assert outd[i].payload_bytes == rd.payload_bytes
            hb = host(blocks[i])
            assert np.array_equal(hb[:rd.payload_bytes], rpay), (call, i)
            assert np.all(hb[rd.payload_bytes:] == 0xAB), "wrote past the payload"
            assert np.array_equal(sse[i], rsse), (call, i)


def test_batch_matches_oracle(G, scenes):
    gsbc, ctx = G
    sel = [0, 1, 2]
    texs = [scenes[i][2] for i in sel]
    descs = [scenes[i][3] for i in sel]
    cap = [int(np.prod(t.shape)) // 4 + 64 for t in texs]
    blocks = [torch.zeros(c, dtype=torch.uint8, device="cuda") for c in cap]
    t = gsbc.default_batch_tuning(wgs_per_cu=2, item_rounds=2, concurrent=1)
    outd, sse = ctx.encode_batch(texs, descs, blocks, tuning=t, want_sse=True)
    for j, i in enumerate(sel):
        pos, sh, _, _, fmt = scenes[i]
        _, rtex, _, _ = O.reorder(pos, sh)
        rpay, roff, rsse = O.encode(rtex, fmt)
        assert np.array_equal(host(blocks[j])[:rpay.size], rpay)
        assert np.array_equal(sse[j], rsse)


def test_batch_replay_reads_current_inputs(G, scenes):
    """Same pointers: the graph is replayed and codes what the buffers hold now."""
    gsbc, ctx = G
    n = 4101
    pos_a, sh_a = synth.make_scene(n, seed=71)
    pos_b, sh_b = synth.make_scene(n, seed=72)
    _, tex, d = ctx.reorder(dev(pos_a), dev(sh_a))
    for k in range(16):
        d.format[k] = 7 if k in (0, 3) else 1
    blocks = [torch.zeros(n * 16, dtype=torch.uint8, device="cuda")]
    outd, _ = ctx.encode_batch([tex], [d], blocks)
    first = host(blocks[0])[:outd[0].payload_bytes].copy()
    _, tex_b, d_b = ctx.reorder(dev(pos_b), dev(sh_b))
    tex.copy_(tex_b)
    outd2, _ = ctx.encode_batch([tex], [d], blocks)
    second = host(blocks[0])[:outd2[0].payload_bytes]
    for k in range(16):
        d_b.format[k] = d.format[k]
    ref, _, _ = _plain(gsbc, ctx, tex_b, d_b)
    assert np.array_equal(second, ref)
    assert not np.array_equal(first, second)


def test_batch_errors(G, scenes):
    gsbc, ctx = G
    tex, d = scenes[1][2], scenes[1][3]
    small = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode_batch([tex], [d], [small])
    assert e.value.status == gsbc.E_BUFFER
    bad = d.copy()
    bad.format[5] = 5   # neither BC1, BC7 nor NONE
    big = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode_batch([tex], [bad], [big])
    assert e.value.status == gsbc.E_ARG
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode_batch([], [], [])
    assert e.value.status == gsbc.E_ARG
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode_batch([tex], [d], [big], tuning=gsbc.default_batch_tuning(bc1_lanes=96))
    assert e.value.status == gsbc.E_ARG
    with pytest.raises(gsbc.GsbcError) as e:
        ctx.encode(tex, bad, fmt=gsbc.FMT_BANDS)
    assert e.value.status == gsbc.E_ARG
