"""Serving loop: encode and decode_eval requests arriving over time.

Requests arrive as a Poisson process.  An encode request codes a scene of N
primitives (reorder, then rate-controlled encode: band 0 BC7, the other
bands chosen per band for an exact mean rate) and leaves its blocks resident
on the device; a decode_eval request evaluates the SH colours of the scene
one earlier encode request produced, at V view directions (random access
into the fixed-size blocks, Sec. I of the paper; colour equation of Sec. II).
A decode waits until its scene is resident.

Continuous batching on one device: a dispatcher admits waiting requests in
arrival order as soon as a slot is free and the request's peak device memory
fits the HBM budget beside the resident scenes and the requests in flight
(least-recently-used scenes that no request is using are evicted to make
room).  Each slot is a worker thread with its own library context and HIP
stream, its scratch arena sized once for the largest admissible request, so
admitted requests overlap on the device and nothing is allocated by the
library mid-stream.  With one slot the same loop is the plain path: one
request at a time, first come first served.

Per request the loop records arrival, admission, start and completion times
and the device time between events on its slot's stream; latency runs from
arrival to completion.  Every kernel decision is independent of what else
runs, so a request's result is the same alone and in the mix; a 64-bit
digest of each sampled result (and the result itself, when asked) lets a
caller check that byte for byte.
"""
import collections
import math
import queue
import threading
import time

import numpy as np
import torch

from . import gsbc, synth

ENCODE, DECODE = "encode", "decode_eval"


class Request:
    __slots__ = ("rid", "kind", "arrival", "n", "v", "offset", "src", "scene", "admitted", "started", "done",
                 "dev_ms", "error", "digest", "output", "blocks_coded", "bytes_out", "mem")

    def __init__(self, rid, kind, arrival, n=0, v=0, offset=0, src=-1):
        self.rid, self.kind, self.arrival, self.n, self.v, self.offset = rid, kind, arrival, n, v, offset
        self.src = src            # decode: rid of the encode request whose scene it reads
        self.scene = None
        self.admitted = self.started = self.done = None
        self.dev_ms = None
        self.error = None
        self.digest = None
        self.output = None
        self.blocks_coded = 0
        self.bytes_out = 0
        self.mem = 0


def make_requests(count, rate_hz, seed=5, n_lo=10_000, n_hi=4_000_000, v_lo=1, v_hi=1024,
                  encode_share=0.7, pool_n=4_000_000):
    """Poisson arrivals at rate_hz; 70/30 encode/decode; N and V log-uniform;
    each decode reads the scene of a uniformly chosen earlier encode."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out, encodes = [], []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        if i == 0 or rng.random() < encode_share:
            n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            off = int(rng.integers(0, pool_n - n + 1))
            out.append(Request(i, ENCODE, t, n=n, offset=off))
            encodes.append(i)
        else:
            v = int(round(math.exp(rng.uniform(math.log(v_lo), math.log(v_hi)))))
            src = encodes[int(rng.integers(0, len(encodes)))]
            out.append(Request(i, DECODE, t, v=v, src=src))
    return out


def payload_bytes(n, rate_bits=6.0):
    """Coded bytes of an n-primitive scene at the rate (band streams 16-byte
    aligned: k + 1 BC7 streams of 16 B per block, 15 - k BC1 of 8 B)."""
    nblk = (n + 15) // 16
    k = int(4 * rate_bits - 17)
    return (k + 1) * 16 * nblk + (15 - k) * ((8 * nblk + 15) // 16 * 16)


def encode_bytes(n):
    """Peak device bytes of one encode request beyond its inputs and the
    slot's reserved scratch: permutation, textures and the final blocks
    (before and after trimming to the payload)."""
    npad = (n + 15) // 16 * 16
    return 4 * n + 64 * npad + 16 * npad + payload_bytes(n) + (1 << 20)


def decode_bytes(n, v):
    return 12 * n * v + 12 * v + (1 << 20)


_M64 = (1 << 64) - 1


def _s64(c):
    return c - (1 << 64) if c >= 1 << 63 else c


_K1, _K2, _K3 = _s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB)


def digest(t):
    """64-bit digest of a device tensor's bytes: every 8-byte word is mixed
    with its position by the SplitMix64 finaliser (a bijective, non-linear
    mix) and the mixed words are summed mod 2^64, so unlike a weighted sum no
    pair of changes can cancel by construction.  Chunked to bound scratch."""
    flat = t.reshape(-1).view(torch.uint8)
    n = flat.numel()
    pad = (-n) % 8
    if pad:
        flat = torch.cat([flat, torch.zeros(pad, dtype=torch.uint8, device=flat.device)])
    words = flat.view(torch.int64)
    h = 0
    chunk = 1 << 25
    for s in range(0, words.numel(), chunk):
        w = words[s:s + chunk]
        z = torch.arange(s, s + w.numel(), device=w.device, dtype=torch.int64) * _K1 + w
        z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _K2
        z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _K3
        z = z ^ ((z >> 31) & ((1 << 33) - 1))
        h = (h + int(z.sum().item())) & _M64
    return (h ^ n) & _M64


class Scene:
    __slots__ = ("sid", "blocks", "desc", "bytes", "users", "last_use")

    def __init__(self, sid, blocks, desc):
        self.sid, self.blocks, self.desc = sid, blocks, desc
        self.bytes = blocks.numel()
        self.users = 0
        self.last_use = time.perf_counter()


class Server:
    def __init__(self, pool_pos, pool_sh, slots=4, hbm_budget=200e9, rate_bits=6.0, device=0,
                 digest_ids=None, keep_ids=(), dirs_seed=11, n_max=4_000_000, v_max=1024):
        self.pool_pos, self.pool_sh = pool_pos, pool_sh
        self.budget = float(hbm_budget)
        self.rate_bits = rate_bits
        self.device = torch.device("cuda", device)
        self.digest_ids = digest_ids       # request ids to digest (None: all)
        self.keep_ids = set(keep_ids)      # request ids whose result is kept on the request
        self.dirs_seed = dirs_seed
        self.scenes = collections.OrderedDict()   # sid (= rid of its encode) -> Scene, LRU order
        self.finished = {}                         # rid -> Request, for decodes' sources
        self.inflight = 0
        self.lock = threading.Lock()
        self.jobs = queue.Queue()
        self.results = queue.Queue()
        self.workers = []
        self.evicted = 0
        # contexts are created here (errors surface at once), each with its
        # scratch sized for the largest admissible request; each is then used
        # by its own worker thread only
        self.slots = []
        for k in range(slots):
            stream = torch.cuda.Stream(self.device)
            ctx = gsbc.Context(self.device.index, stream=stream)
            ctx.reserve(n_max, v_max)
            self.slots.append((stream, ctx))
        self.growths0 = sum(ctx.arena_info()[1] for _, ctx in self.slots)
        for k in range(slots):
            th = threading.Thread(target=self._worker, args=(k,), daemon=True)
            th.start()
            self.workers.append(th)

    def arena_growths(self):
        """Scratch growths of the slots' contexts since they were reserved."""
        return sum(ctx.arena_info()[1] for _, ctx in self.slots) - self.growths0

    # ---------------------------------------------------------------- memory
    def resident_bytes(self):
        return sum(s.bytes for s in self.scenes.values())

    def _fits(self, need):
        return self.resident_bytes() + self.inflight + need <= self.budget

    def _make_room(self, need):
        """Evict idle scenes (least recently used first) until `need` fits."""
        if self._fits(need):
            return True
        for sid in list(self.scenes):
            if self._fits(need):
                break
            sc = self.scenes[sid]
            if sc.users == 0:
                del self.scenes[sid]
                self.evicted += 1
        return self._fits(need)

    # ---------------------------------------------------------------- workers
    def _worker(self, k):
        torch.cuda.set_device(self.device)
        stream, ctx = self.slots[k]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        while True:
            job = self.jobs.get()
            if job is None:
                ctx.close()
                return
            req, scene = job
            req.started = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    e0.record(stream)
                    if req.kind == ENCODE:
                        out = self._run_encode(ctx, req)
                    else:
                        out = self._run_decode(ctx, req, scene)
                    e1.record(stream)
                stream.synchronize()
                req.done = time.perf_counter()   # completion; digests are not part of it
                req.dev_ms = e0.elapsed_time(e1)
                res = out[0] if req.kind == ENCODE else out
                if self.digest_ids is None or req.rid in self.digest_ids:
                    with torch.cuda.stream(stream):
                        req.digest = digest(res)
                if req.rid in self.keep_ids:
                    req.output = res
                out = out if req.kind == ENCODE else None
                res = None   # a decode output is released before its memory is
                self.results.put((req, out))
            except Exception as e:   # reported per request; the loop goes on
                req.error = repr(e)
                req.done = time.perf_counter()
                self.results.put((req, None))

    def _run_encode(self, ctx, req):
        pos = self.pool_pos[req.offset:req.offset + req.n]
        sh = self.pool_sh[req.offset:req.offset + req.n]
        _, tex, d = ctx.reorder(pos, sh)
        blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_AUTO, rate=self.rate_bits)
        blocks = blocks[:d2.payload_bytes].clone()   # keep only the payload resident
        req.blocks_coded = 16 * d2.blocks_per_stream
        return blocks, d2

    def _run_decode(self, ctx, req, scene):
        dirs = torch.from_numpy(synth.make_dirs(req.v, seed=self.dirs_seed + req.rid)).to(self.device)
        out = ctx.decode_eval(scene.blocks, scene.desc, dirs)
        req.bytes_out = out.numel() * 4
        return out

    # ---------------------------------------------------------------- dispatch
    def _decode_source(self, req):
        """The finished encode request a decode reads, or None while that
        encode has not finished."""
        return self.finished.get(req.src)

    def run(self, requests, time_scale=1.0, poll_s=2e-4, on_done=None, deadline_s=None):
        """Serve `requests` (arrival times in seconds from start).  A request
        still waiting for admission `deadline_s` after its arrival is dropped
        with an error (the watchdog).  Returns the finished requests."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = []
        free_slots = len(self.workers)
        done = []
        t0 = time.perf_counter()
        total = len(requests)

        def finish(req, err):
            req.error = err
            req.done = time.perf_counter()
            self.finished[req.rid] = req
            done.append(req)

        while len(done) < total:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival * time_scale <= now:
                waiting.append(pending.popleft())
            if deadline_s is not None:
                for req in [r for r in waiting if now - r.arrival * time_scale > deadline_s]:
                    waiting.remove(req)
                    finish(req, "deadline passed before admission")
            # admit in arrival order while slots and memory allow
            i = 0
            while free_slots > 0 and i < len(waiting):
                req = waiting[i]
                with self.lock:
                    sc = None
                    if req.kind == DECODE:
                        src = self._decode_source(req)
                        if src is None:        # its scene is still being coded
                            i += 1
                            continue
                        need = decode_bytes(src.n, req.v)
                        sc = self.scenes.get(req.src)
                        err = ("source scene unavailable" if src.error else
                               "request exceeds the HBM budget" if need > self.budget else
                               "source scene evicted" if sc is None else None)
                        if err:
                            waiting.pop(i)
                            finish(req, err)
                            continue
                        sc.users += 1          # the scene it reads is not evicted to make room
                    else:
                        need = encode_bytes(req.n)
                    if need > self.budget or not self._make_room(need):
                        if sc is not None:
                            sc.users -= 1
                        if need > self.budget:
                            waiting.pop(i)
                            finish(req, "request exceeds the HBM budget")
                            continue
                        i += 1
                        continue
                    self.inflight += need
                    req.mem = need
                    if sc is not None:
                        sc.last_use = time.perf_counter()
                        self.scenes.move_to_end(sc.sid)
                        req.scene = sc.sid
                waiting.pop(i)
                req.admitted = time.perf_counter()
                free_slots -= 1
                self.jobs.put((req, sc))
            # completions
            got = False
            while True:
                try:
                    req, out = self.results.get_nowait()
                except queue.Empty:
                    break
                got = True
                free_slots += 1
                with self.lock:
                    self.inflight -= req.mem
                    if req.kind == DECODE and req.scene in self.scenes:
                        self.scenes[req.scene].users -= 1
                    if req.kind == ENCODE and out is not None:
                        self.scenes[req.rid] = Scene(req.rid, out[0], out[1])
                        req.scene = req.rid
                    self.finished[req.rid] = req
                if on_done:
                    on_done(req)
                done.append(req)
            if not got:
                time.sleep(poll_s)
        self.t_elapsed = time.perf_counter() - t0
        self.t0 = t0
        return done

    def close(self):
        for _ in self.workers:
            self.jobs.put(None)
        for th in self.workers:
            th.join()
        self.workers = []
        self.slots = []

    # ---------------------------------------------------------------- solo replay
    def run_alone(self, req):
        """Run one finished request again with nothing else on the device;
        returns (digest, result).  A decode reads the same resident scene."""
        torch.cuda.synchronize()
        ctx = gsbc.Context(self.device.index)
        try:
            r = Request(req.rid, req.kind, 0.0, n=req.n, v=req.v, offset=req.offset, src=req.src)
            if req.kind == ENCODE:
                res = self._run_encode(ctx, r)[0]
            else:
                res = self._run_decode(ctx, r, self.scenes[req.scene])
            torch.cuda.synchronize()
            return digest(res), res
        finally:
            ctx.close()


def _pct(a, q):
    return round(float(np.percentile(a, q)), 3) if len(a) else None


def summarize(done, t_elapsed, t0):
    """Latency percentiles (arrival -> completion), their parts, throughput."""
    ok = [r for r in done if r.error is None]

    def lat(rs):
        return np.array([(r.done - (t0 + r.arrival)) * 1e3 for r in rs])

    enc = [r for r in ok if r.kind == ENCODE]
    dec = [r for r in ok if r.kind == DECODE]
    queue_ms = np.array([(r.admitted - (t0 + r.arrival)) * 1e3 for r in ok])
    dispatch_ms = np.array([(r.started - r.admitted) * 1e3 for r in ok])
    run_ms = np.array([(r.done - r.started) * 1e3 for r in ok])
    dev_ms = np.array([r.dev_ms for r in ok])
    blocks = sum(r.blocks_coded for r in enc)
    by = sum(r.bytes_out for r in dec)
    la = lat(ok)
    return {"requests": len(done), "errors": sum(r.error is not None for r in done),
            "p50_ms": _pct(la, 50), "p99_ms": _pct(la, 99), "mean_ms": round(float(la.mean()), 3) if len(la) else None,
            "encode_p50_ms": _pct(lat(enc), 50), "encode_p99_ms": _pct(lat(enc), 99),
            "decode_p50_ms": _pct(lat(dec), 50), "decode_p99_ms": _pct(lat(dec), 99),
            # where the time goes: waiting for a slot or memory (arrival ->
            # admission), hand-over to the slot's thread, and the slot's run
            # (start -> completion: host work plus the device time below,
            # which also counts time its kernels shared the GPU)
            "breakdown_ms": {"queue_p50": _pct(queue_ms, 50), "queue_p99": _pct(queue_ms, 99),
                             "queue_mean": round(float(queue_ms.mean()), 3) if len(ok) else None,
                             "dispatch_p50": _pct(dispatch_ms, 50),
                             "run_p50": _pct(run_ms, 50), "run_p99": _pct(run_ms, 99),
                             "run_mean": round(float(run_ms.mean()), 3) if len(ok) else None,
                             "device_p50": _pct(dev_ms, 50), "device_p99": _pct(dev_ms, 99)},
            "elapsed_s": round(t_elapsed, 3), "encode_mblocks_s": round(blocks / t_elapsed / 1e6, 3),
            "decode_gb_s": round(by / t_elapsed / 1e9, 3)}
