"""Serving loop: encode and decode_eval requests arriving over time.

Requests arrive as a Poisson process.  An encode request codes a scene of N
primitives (reorder, then rate-controlled encode: band 0 BC7, the other
bands chosen per band for an exact mean rate) and leaves its blocks resident
on the device; a decode_eval request evaluates the SH colours of a resident
scene at V view directions (random access into the fixed-size blocks,
Sec. I of the paper; colour equation of Sec. II).

Continuous batching on one device: a dispatcher admits waiting requests in
arrival order as soon as a slot is free and the request's peak device memory
fits the HBM budget beside the resident scenes and the requests in flight
(least-recently-used scenes that no request is using are evicted to make
room).  Each slot is a worker thread with its own library context and HIP
stream, so admitted requests overlap on the device.  Latency is measured
from arrival to completion.  Every kernel decision is independent of what
else runs, so a request's result is the same alone and in the mix; the
fingerprints recorded per request let a caller check that.
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
    __slots__ = ("rid", "kind", "arrival", "n", "v", "offset", "scene", "admitted", "started", "done",
                 "error", "fingerprint", "blocks_coded", "bytes_out", "mem")

    def __init__(self, rid, kind, arrival, n=0, v=0, offset=0):
        self.rid, self.kind, self.arrival, self.n, self.v, self.offset = rid, kind, arrival, n, v, offset
        self.scene = None
        self.admitted = self.started = self.done = None
        self.error = None
        self.fingerprint = None
        self.blocks_coded = 0
        self.bytes_out = 0
        self.mem = 0


def make_requests(count, rate_hz, seed=5, n_lo=10_000, n_hi=4_000_000, v_lo=1, v_hi=1024,
                  encode_share=0.7, pool_n=4_000_000):
    """Poisson arrivals at rate_hz; 70/30 encode/decode; N and V log-uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        if i == 0 or rng.random() < encode_share:
            n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            off = int(rng.integers(0, pool_n - n + 1))
            out.append(Request(i, ENCODE, t, n=n, offset=off))
        else:
            v = int(round(math.exp(rng.uniform(math.log(v_lo), math.log(v_hi)))))
            out.append(Request(i, DECODE, t, v=v))
    return out


def encode_bytes(n):
    """Peak device bytes of one encode request beyond its inputs: permutation,
    textures, final blocks and the context's scratch (both candidate
    payloads, run tables, BC7 keys)."""
    npad = (n + 15) // 16 * 16
    nblk = npad // 16
    return 4 * n + 64 * npad + 16 * npad + (16 * (8 * nblk + 16) + 16 * 16 * nblk) + 8 * 16 * (nblk + 256) + (1 << 20)


def decode_bytes(n, v):
    return 12 * n * v + 12 * v + 16 * 4 * v + (1 << 20)


def fingerprint(t):
    """Order-sensitive 64-bit fingerprint of a device tensor's bytes (chunked)."""
    flat = t.reshape(-1).view(torch.uint8)
    n = flat.numel()
    n4 = n // 4 * 4
    words = flat[:n4].view(torch.int32)
    h = 0
    chunk = 1 << 26
    for s in range(0, words.numel(), chunk):
        w = words[s:s + chunk].to(torch.int64)
        idx = torch.arange(s, s + w.numel(), device=w.device, dtype=torch.int64)
        h = (h * 1_000_003 + int(((w + 0x9E3779B9) * (idx % 65_521 + 1)).sum().item())) & ((1 << 64) - 1)
    tail = flat[n4:].to(torch.int64).sum().item() if n4 < n else 0
    return (h ^ (tail * 0x100000001B3)) & ((1 << 64) - 1)


class Scene:
    __slots__ = ("sid", "blocks", "desc", "bytes", "users", "last_use")

    def __init__(self, sid, blocks, desc):
        self.sid, self.blocks, self.desc = sid, blocks, desc
        self.bytes = blocks.numel()
        self.users = 0
        self.last_use = time.perf_counter()


class Server:
    def __init__(self, pool_pos, pool_sh, slots=4, hbm_budget=200e9, rate_bits=6.0, device=0,
                 fingerprint_ids=None, dirs_seed=11):
        self.pool_pos, self.pool_sh = pool_pos, pool_sh
        self.budget = float(hbm_budget)
        self.rate_bits = rate_bits
        self.device = torch.device("cuda", device)
        self.fp_ids = fingerprint_ids      # request ids to fingerprint (None: all)
        self.dirs_seed = dirs_seed
        self.scenes = collections.OrderedDict()   # sid -> Scene, LRU order
        self.inflight = 0
        self.lock = threading.Lock()
        self.jobs = queue.Queue()
        self.results = queue.Queue()
        self.workers = []
        self.evicted = 0
        self.sid_next = 0
        self.rng = np.random.Generator(np.random.PCG64(1234))   # decode requests' scene choice
        # contexts are created here (errors surface at once); each is then
        # used by its own worker thread only
        self.slots = []
        for k in range(slots):
            stream = torch.cuda.Stream(self.device)
            self.slots.append((stream, gsbc.Context(self.device.index, stream=stream)))
        for k in range(slots):
            th = threading.Thread(target=self._worker, args=(k,), daemon=True)
            th.start()
            self.workers.append(th)

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
        while True:
            job = self.jobs.get()
            if job is None:
                ctx.close()
                return
            req, scene = job
            req.started = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    if req.kind == ENCODE:
                        out = self._run_encode(ctx, req)
                    else:
                        out = self._run_decode(ctx, req, scene)
                stream.synchronize()
                req.done = time.perf_counter()   # completion; fingerprinting is not part of it
                if self.fp_ids is None or req.rid in self.fp_ids:
                    req.fingerprint = fingerprint(out[0] if req.kind == ENCODE else out)
                    stream.synchronize()
                res = out if req.kind == ENCODE else None
                out = None   # a decode output is released before its memory is
                self.results.put((req, res))
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
    def run(self, requests, time_scale=1.0, poll_s=2e-4, on_done=None, deadline_s=None):
        """Serve `requests` (arrival times in seconds from start).  A request
        still waiting for admission `deadline_s` after its arrival is dropped
        with an error (the watchdog).  Returns the finished requests."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = []
        free_slots = len(self.workers)
        done = []
        rng = self.rng
        t0 = time.perf_counter()
        total = len(requests)
        while len(done) < total:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival * time_scale <= now:
                waiting.append(pending.popleft())
            if deadline_s is not None:
                for req in [r for r in waiting if now - r.arrival * time_scale > deadline_s]:
                    waiting.remove(req)
                    req.error = "deadline passed before admission"
                    req.done = time.perf_counter()
                    done.append(req)
            # admit in arrival order while slots and memory allow
            i = 0
            while free_slots > 0 and i < len(waiting):
                req = waiting[i]
                with self.lock:
                    if req.kind == DECODE:
                        if not self.scenes:
                            i += 1
                            continue
                        keys = list(self.scenes)
                        sc = self.scenes[keys[int(rng.integers(0, len(keys)))]]
                        need = decode_bytes(sc.desc.n_prims, req.v)
                    else:
                        sc = None
                        need = encode_bytes(req.n)
                    if sc is not None:
                        sc.users += 1          # the scene it reads is not evicted to make room
                    if need > self.budget or not self._make_room(need):
                        if sc is not None:
                            sc.users -= 1
                        if need > self.budget:
                            req.error = "request exceeds the HBM budget"
                            waiting.pop(i)
                            req.done = time.perf_counter()
                            done.append(req)
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
                        sid = self.sid_next
                        self.sid_next += 1
                        self.scenes[sid] = Scene(sid, out[0], out[1])
                        req.scene = sid
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
        """Run one finished request again with nothing else on the device and
        return its fingerprint (decode requests reuse the scene they read)."""
        r = Request(req.rid, req.kind, 0.0, n=req.n, v=req.v, offset=req.offset)
        res = self.run([r]) if req.kind == ENCODE else None
        if req.kind == DECODE:
            sc = self.scenes[req.scene]
            ctx = gsbc.Context(self.device.index)
            out = self._run_decode(ctx, r, sc)
            torch.cuda.synchronize()
            fp = fingerprint(out)
            ctx.close()
            return fp
        return res[0].fingerprint


def summarize(done, t_elapsed, t0):
    lat = np.array([(r.done - (t0 + r.arrival)) * 1e3 for r in done if r.error is None])
    enc = [r for r in done if r.kind == ENCODE and r.error is None]
    dec = [r for r in done if r.kind == DECODE and r.error is None]
    blocks = sum(r.blocks_coded for r in enc)
    by = sum(r.bytes_out for r in dec)

    def pct(a, q):
        return round(float(np.percentile(a, q)), 3) if len(a) else None
    lat_e = np.array([(r.done - (t0 + r.arrival)) * 1e3 for r in enc])
    lat_d = np.array([(r.done - (t0 + r.arrival)) * 1e3 for r in dec])
    return {"requests": len(done), "errors": sum(r.error is not None for r in done),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "encode_p50_ms": pct(lat_e, 50), "encode_p99_ms": pct(lat_e, 99),
            "decode_p50_ms": pct(lat_d, 50), "decode_p99_ms": pct(lat_d, 99),
            "elapsed_s": round(t_elapsed, 3), "encode_mblocks_s": round(blocks / t_elapsed / 1e6, 3),
            "decode_gb_s": round(by / t_elapsed / 1e9, 3)}
