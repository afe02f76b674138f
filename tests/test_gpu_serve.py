"""GPU: the serving loop.  Requests of mixed kinds and sizes overlap on the
device through several slots; each result must be the same as the request
run alone afterwards (bit-identical blocks and colours), the HBM budget must
hold requests back or reject them without crashing, and the deadline
watchdog must drop requests that wait too long."""
import sys

import numpy as np
import pytest

from paper_2607_14513_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POOL = 200_000


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pool():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pos, sh = synth.make_scene_device(POOL, seed=5, device="cuda")
    torch.cuda.synchronize()
    return pos, sh


def _reqs(serve, count, rate, seed, n_hi=60_000, v_hi=96):
    return serve.make_requests(count, rate, seed=seed, n_lo=1_000, n_hi=n_hi, v_lo=1, v_hi=v_hi, pool_n=POOL)


def test_mix_equals_alone(pool):
    from paper_2607_14513_amd import serve
    reqs = _reqs(serve, 40, 3000.0, seed=21)
    srv = serve.Server(*pool, slots=3, hbm_budget=4e9, keep_ids={r.rid for r in reqs}, n_max=POOL, v_max=96)
    try:
        say("serve mix", len(reqs))
        done = srv.run(reqs)
        assert len(done) == len(reqs)
        assert all(r.error is None for r in done), [r.error for r in done if r.error]
        assert srv.inflight == 0
        assert srv.arena_growths() == 0      # every slot's scratch was sized up front
        kinds = {r.kind for r in done}
        assert kinds == {serve.ENCODE, serve.DECODE}
        overlapped = sum(1 for a in done for b in done
                         if a.rid < b.rid and a.started < b.done and b.started < a.done)
        say("overlapping pairs", overlapped)
        for r in sorted(done, key=lambda r: r.rid):
            dg, alone = srv.run_alone(r)
            assert torch.equal(alone, r.output), (r.rid, r.kind, r.n, r.v)     # byte for byte
            assert dg == r.digest, (r.rid, r.kind)
            if r.kind == serve.DECODE:
                assert r.output.shape == (r.v, srv.finished[r.src].n, 3)
    finally:
        srv.close()


def test_digest_sees_every_byte():
    """The result digest changes with any single byte, and with two changes
    that would cancel in a position-weighted sum."""
    from paper_2607_14513_amd import serve
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.integers(0, 256, 1 << 20, dtype=np.uint8)).cuda()
    h = serve.digest(a)
    for i in (0, 1, 12345, (1 << 20) - 1):
        b = a.clone()
        b[i] ^= 1
        assert serve.digest(b) != h
    b = a.clone()
    b[8], b[16] = a[16], a[8]      # swap two words' first bytes
    if not torch.equal(a, b):
        assert serve.digest(b) != h
    assert serve.digest(a[:-3]) != h


def test_budget_admission_and_eviction(pool):
    from paper_2607_14513_amd import serve
    reqs = serve.make_requests(32, 5000.0, seed=22, n_lo=20_000, n_hi=40_000, v_lo=1, v_hi=16, pool_n=POOL)
    # one oversized decode (needs more than the whole budget) among them
    reqs.append(serve.Request(len(reqs), serve.DECODE, reqs[-1].arrival + 1e-3, v=4000, src=reqs[0].rid))
    budget = 6e6
    enc = [r for r in reqs if r.kind == serve.ENCODE]
    # every encode fits the budget alone, but their resident payloads
    # together do not: since all encodes must succeed, idle scenes have to be
    # evicted whatever the timing (payload at 6 bits/texel: 8 BC7 streams of
    # 16 B and 8 BC1 streams of 8 B per block, each stream 16-byte aligned)
    def payload(n):
        nblk = (n + 15) // 16
        return 8 * 16 * nblk + 8 * ((8 * nblk + 15) // 16 * 16)
    assert max(serve.encode_bytes(r.n) for r in enc) <= budget < sum(payload(r.n) for r in enc)
    srv = serve.Server(*pool, slots=2, hbm_budget=budget, n_max=40_000, v_max=16)
    try:
        done = srv.run(reqs)
        assert len(done) == len(reqs)
        errs = [r for r in done if r.error]
        assert any("budget" in r.error for r in errs)
        assert all(r.error is None for r in done if r.kind == serve.ENCODE)
        assert srv.inflight == 0
        assert srv.resident_bytes() <= budget
        assert srv.evicted > 0
    finally:
        srv.close()


def test_deadline_watchdog(pool):
    from paper_2607_14513_amd import serve
    reqs = _reqs(serve, 12, 1e6, seed=23, n_hi=40_000)
    srv = serve.Server(*pool, slots=1, hbm_budget=4e9, n_max=POOL, v_max=96)
    try:
        done = srv.run(reqs, deadline_s=0.002)
        assert len(done) == len(reqs)
        dropped = [r for r in done if r.error and "deadline" in r.error]
        assert dropped
        assert any(r.error is None for r in done)
        assert srv.inflight == 0
    finally:
        srv.close()
