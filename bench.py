#!/usr/bin/env python3
"""Benchmark of the SH BC1/BC7 coding path on one MI355X.

One step = the whole path over one synthetic scene already resident in HBM:
  reorder (range, keys, stable radix sort, gather + pack)
  -> encode every band in BC1 and in BC7 and keep the 6 bits/texel choice
  -> random-access decode + SH evaluation at 64 view directions.
Workload: 1,048,576 primitives (32 position clusters, 64-component DC colour
mixture, Laplacian higher bands; seed 2), i.e. 1,048,576 blocks per format.

Prints one JSON line.  `value` = blocks encoded per step (both formats) /
step time, in Mblocks/s.  Also reported:
  roofline            the step's dominant kernel (a BC7 search kernel):
                      algorithmic integer ops per launch / its average launch
                      time (HIP events the library records on its stream),
                      against the VALU peak;
  kernels_ms_per_step per-kernel device times of the same step from extra
                      passes with the library's kernel timing on, which runs
                      the encoder's kernels one after another (the timed steps
                      overlap BC1 with the BC7 bucketing and emit kernels);
  valu_issue          the BC7 search and BC1 encoders' VALU instructions per
                      launch (SQ_INSTS_VALU of the committed rocprofv3 pass)
                      over the live launch time, against one wave64
                      instruction per SIMD every 4 cycles at 2.4 GHz (1.0 =
                      every issue slot used; the 4-cycle model is not exact
                      for every instruction, so it can read slightly above 1);
  roofline_decode_eval  decode + SH evaluation of 3,145,728 primitives at
                      1,024 directions: bytes written+read per launch / time,
                      against 8 TB/s; with the view decode and the fused
                      colour stage (tile blend at 1920x1088) of that scene;
  cpu_baseline        the CPU oracle on a bounded sample of the same step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 4 * 16 * 2.4e9        # integer lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4    # wave64 VALU instructions/s (4 cycles each per SIMD)
HBM_PEAK = 8.0e12                        # bytes/s
# VALU issue slots (lane-instructions) that one exact texel x palette-entry
# distance comparison needs at the least on gfx950: one v_dot2 for two
# channels, one 24-bit multiply-add for the third channel plus the entry's
# constant, and half a v_min3 for the running minimum.  A plain scalar form
# takes about 8 (3 sub, 3 mul, 2 add); the issue-slot floor is what bounds
# the kernel, so the fraction below is the share of peak VALU issue spent on
# that irreducible work.
OPS_PER_EVAL = 2.5
# Algorithmic work per block of the BC7 search kernels: texel x palette-entry
# distance evaluations of the candidates each kernel covers (initial fit and
# least-squares refit, every p-bit choice) x OPS_PER_EVAL.
ALGO_OPS = {
    "bc7_search_2subset": 3 * 32_768 * OPS_PER_EVAL,            # modes 1, 3, 7
    "bc7_search_3subset": (16_384 + 8_192) * OPS_PER_EVAL,     # modes 0, 2
    "bc7_search_1subset": (3_072 + 1_024 + 2_048) * OPS_PER_EVAL,  # modes 4, 5, 6
}
# one launch over every group (work items per group, or all groups per block)
ALGO_OPS["bc7_search_items"] = ALGO_OPS["bc7_search_all"] = sum(ALGO_OPS.values())
# The evaluations the search actually executes: a 3-subset mask that recurs
# across partitions is fitted once per mode and its SSE reused, so mode 2
# fits 140 distinct masks of its 192 (5,984 of 8,192 evaluations) and mode 0
# 36 of 48 (12,288 of 16,384).  The refit's evaluation is also skipped when
# its normal equations are singular (data-dependent, not counted here).
EXECUTED_EVALS = 3 * 32_768 + 12_288 + 5_984 + 3_072 + 1_024 + 2_048
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_encode_step_1M_and_decode_eval_3M.json")


def profiled(name, field="bytes"):
    """A per-launch figure of kernel `name` from the committed rocprofv3
    counter summary: "bytes" = HBM bytes (FETCH_SIZE and WRITE_SIZE scaled by
    a 1 GiB copy), "valu_insts" = SQ_INSTS_VALU.  None when there is none or
    the kernel's source changed since."""
    if not os.path.exists(TRAFFIC):
        return None
    ent = json.load(open(TRAFFIC)).get(name)
    if not ent or field not in ent:
        return None
    src = os.path.join(ROOT, ent["source"])
    if not os.path.exists(src) or hashlib.sha1(open(src, "rb").read()).hexdigest() != ent["source_sha1"]:
        return None
    return ent[field]


def traffic_bytes(name):
    return profiled(name, "bytes")


def progress(msg):
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def med_min(ts, scale=1.0, nd=4):
    """Median and minimum of repeated timings (scaled, rounded)."""
    return {"median": round(float(np.median(ts)) * scale, nd), "min": round(float(np.min(ts)) * scale, nd)}


def kernel_ms(ctx, name, call, reps):
    """Device time of the kernel(s) `name` (one name or a tuple, summed) in
    each of `reps` calls (the library's HIP events on its stream), ms."""
    names = (name,) if isinstance(name, str) else tuple(name)
    ctx.profile(True)
    ctx.profile_read()
    ts = []
    for _ in range(reps):
        call()
        k = ctx.profile_read()
        ts.append(sum(k[nm][1] / k[nm][0] for nm in names))
    ctx.profile(False)
    return ts


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rate", type=float, default=6.0)
    ap.add_argument("--dirs", type=int, default=64)
    ap.add_argument("--no-large", action="store_true", help="skip the 3,145,728-primitive decode_eval leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (for counter scaling)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-scene batched-encode leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-degrees", action="store_true", help="skip the degree-class (variable bands) leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--batch-scenes", type=int, default=64)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by block ranges, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_14513_amd import gsbc, synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    cfg = synth.CONFIGS["mid"]
    n, V, rate = cfg["n"], args.dirs, args.rate
    pos, sh = synth.make_scene(n, cfg["clusters"], cfg["comps"], cfg["seed"])
    dirs = synth.make_dirs(V, seed=cfg["seed"])
    nblk = (n + 15) // 16

    with torch.cuda.stream(stream):
        if args.copy_calibration:
            a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
            a.fill_(1.0)
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        ctx = gsbc.Context(0, stream=stream)
        pos_d = torch.from_numpy(pos).to(dev)
        sh_d = torch.from_numpy(sh).to(dev)
        dirs_d = torch.from_numpy(dirs).to(dev)
        _, cap, _ = gsbc.query_sizes(n)
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        tex = torch.empty((16, nblk, 16, 4), dtype=torch.uint8, device=dev)
        blocks = torch.empty(cap, dtype=torch.uint8, device=dev)
        out = torch.empty((V, n, 3), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()

        def step(ev=None):
            if ev:
                ev[0].record(stream)
            _, _, d = ctx.reorder(pos_d, sh_d, out=(perm, tex))
            if ev:
                ev[1].record(stream)
            _, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_AUTO, rate=rate, blocks=blocks)
            if ev:
                ev[2].record(stream)
            ctx.decode_eval(blocks, d2, dirs_d, out=out)
            if ev:
                ev[3].record(stream)
            return d2

        for _ in range(args.warmup):
            d2 = step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            d2 = step(evs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])] for e in evs])
        ms_step = wall * 1e3 / args.steps
        blocks_per_step = 2 * 16 * nblk
        value = blocks_per_step / (ms_step * 1e-3) / 1e6

        progress(f"timed {args.steps} steps: {ms_step:.3f} ms per step")
        # ---- per-kernel device times of the same step (HIP events the library
        # records on its stream around every launch), read back step by step
        ctx.profile(True)
        ctx.profile_read()
        nprof = max(3, args.steps)
        per_run = []
        for _ in range(nprof):
            step()
            per_run.append(ctx.profile_read())
        ctx.profile(False)
        kern = {}
        for r in per_run:
            for k, (cnt, ms) in r.items():
                c0, m0 = kern.get(k, (0, 0.0))
                kern[k] = (c0 + cnt, m0 + ms)
        per_step = {k: v[1] / nprof for k, v in kern.items()}
        dom = max(per_step, key=per_step.get)
        launches = kern[dom][0] / nprof
        dom_s = per_step[dom] / launches * 1e-3                     # average launch, s
        dom_launch_ms = [r[dom][1] / r[dom][0] for r in per_run if dom in r]
        units = 16 * nblk                                           # blocks per launch
        work = ALGO_OPS.get(dom)
        traffic = traffic_bytes(dom)
        roof = {"kernel": dom, "bound": "alu", "achieved": work * units / dom_s / 1e12 if work else None,
                "peak": VALU_PEAK / 1e12, "unit": "Tops/s",
                "frac": work * units / dom_s / VALU_PEAK if work else None, "traffic": traffic,
                "launch_ms": round(dom_s * 1e3, 4), "launch_ms_median": round(float(np.median(dom_launch_ms)), 4),
                "launch_ms_min": round(float(np.min(dom_launch_ms)), 4),
                "algorithmic_ops_per_block": work, "blocks_per_launch": units}
        if dom in ("bc7_search_items", "bc7_search_all"):
            # the same floor over the evaluations the kernel executes
            roof["executed_ops_per_block"] = EXECUTED_EVALS * OPS_PER_EVAL
            roof["frac_executed"] = EXECUTED_EVALS * OPS_PER_EVAL * units / dom_s / VALU_PEAK

        # ---- counter-measured VALU issue utilisation of the encoders: the
        # committed SQ_INSTS_VALU count of a launch over the live launch time
        valu = {}
        for name in ("bc7_search_items", "bc1_encode"):
            insts = profiled(name, "valu_insts")
            if name in kern and insts:
                t = per_step[name] / (kern[name][0] / nprof) * 1e-3
                valu[name] = {"valu_insts_per_launch": insts, "launch_ms": round(t * 1e3, 4),
                              "issue_busy": round(insts / t / VALU_ISSUE_PEAK, 4)}

        progress("per-kernel times done")
        # ---- whole-format encode rates (every band in one format)
        d7 = d2.copy()
        rates = {}
        for fmt, name in ((gsbc.FMT_BC7, "bc7"), (gsbc.FMT_BC1, "bc1")):
            ts = []
            for i in range(max(3, args.steps)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ctx.encode(tex, d7, fmt=fmt, blocks=blocks)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            rates[name] = 16 * nblk / float(np.median(ts)) / 1e6
            rates[name + "_ms"] = med_min(ts, 1e3)

        # ---- per-band PSNR of the decoded coefficient texels (sorted order and
        # the input order), 10 log10(255^2 / MSE) over all RGB texels
        def band_psnr(texd, fmt):
            b, dd, _ = ctx.encode(texd, d7, fmt=fmt, blocks=blocks)
            dec = ctx.decode(b, dd)
            diff = dec[..., :3].to(torch.int32) - texd[..., :3].to(torch.int32)
            mse = (diff * diff).sum(dim=(1, 2, 3)).double().cpu().numpy() / (dd.n_pad * 3)
            return [round(float(10 * np.log10(255.0 ** 2 / m)), 2) if m > 0 else None for m in mse]

        _, tex_id, d_id = ctx.reorder(pos_d, sh_d, params=gsbc.default_params(order=1))
        psnr = {"bc1_sorted": band_psnr(tex, gsbc.FMT_BC1), "bc7_sorted": band_psnr(tex, gsbc.FMT_BC7),
                "bc1_input_order": band_psnr(tex_id, gsbc.FMT_BC1),
                "bc7_input_order": band_psnr(tex_id, gsbc.FMT_BC7)}
        del tex_id

        progress("format rates and PSNR done")
        # ---- the arrangements of Table I (Figs. SetupA, SetupB, SetupD) on this
        # scene: PSNR of the decoded texels over all bands and slots, and the
        # coded bytes per primitive
        def arrangement_row(label, arr, order, fmts):
            _, tx, dd = ctx.reorder(pos_d, sh_d, params=gsbc.default_params(arrangement=arr, order=order))
            for k, f in enumerate(fmts):
                dd.format[k] = f
            b, d3, _ = ctx.encode(tx, dd, fmt=gsbc.FMT_BANDS, blocks=blocks)
            dec = ctx.decode(b, d3)
            diff = dec[..., :3].to(torch.int32) - tx[..., :3].to(torch.int32)
            mse = float((diff * diff).sum(dtype=torch.float64).item()) / (d3.n_pad * 48)
            return {"arrangement": label, "psnr_db": round(float(10 * np.log10(255.0 ** 2 / mse)), 2),
                    "bytes_per_primitive": round(d3.payload_bytes / n, 3)}

        arrangements = []
        for label, arr, order, fmts in (
                ("SetupA: BC1", 1, 1, [1]), ("SetupA: BC7", 1, 1, [7]),
                ("SetupB: BC7 + 3 BC1, input order", 2, 1, [7, 1, 1, 1]),
                ("SetupB: BC7 + 3 BC1, sorted", 2, 0, [7, 1, 1, 1]),
                ("SetupD: 16 BC1, input order", 0, 1, [1] * 16), ("SetupD: 16 BC1, sorted", 0, 0, [1] * 16),
                ("SetupD: BC7 + 15 BC1, input order", 0, 1, [7] + [1] * 15),
                ("SetupD: BC7 + 15 BC1, sorted", 0, 0, [7] + [1] * 15),
                ("SetupD: 16 BC7, input order", 0, 1, [7] * 16), ("SetupD: 16 BC7, sorted", 0, 0, [7] * 16)):
            arrangements.append(arrangement_row(label, arr, order, fmts))
        torch.cuda.empty_cache()

        # ---- variable number of bands (degree classes) on a scene of the same
        # size whose primitives use SH degree 0..3 in proportions MIX: classes
        # coded band 0 BC7 + the rest BC1 in one batch, against all 16 bands
        degrees = None
        if not args.no_degrees:
            mix = (0.35, 0.2, 0.15, 0.3)
            posg, shg = synth.make_scene(n, cfg["clusters"], cfg["comps"], cfg["seed"] + 100, degree_mix=mix)
            posg_d, shg_d = torch.from_numpy(posg).to(dev), torch.from_numpy(shg).to(dev)
            del posg, shg
            ctx.reorder_degrees(posg_d, shg_d)                    # warm-up
            t_re = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                permg, counts, texg, descg = ctx.reorder_degrees(posg_d, shg_d)
                e1.record(stream)
                torch.cuda.synchronize()
                t_re.append(e0.elapsed_time(e1))
            live = [L for L in range(4) if counts[L]]
            for L in live:
                for k in range(descg[L].n_streams):
                    descg[L].format[k] = 7 if k == 0 else 1
            bufs = [torch.empty(descg[L].n_pad * 16, dtype=torch.uint8, device=dev) for L in live]
            tx = [texg[L] for L in live]
            dsc = [descg[L] for L in live]
            ctx.encode_batch(tx, dsc, bufs)
            t_cls = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                outd, _ = ctx.encode_batch(tx, dsc, bufs)
                e1.record(stream)
                torch.cuda.synchronize()
                t_cls.append(e0.elapsed_time(e1))
            bytes_cls = sum(d.payload_bytes for d in outd)
            _, tfull, dfull = ctx.reorder(posg_d, shg_d)
            for k in range(16):
                dfull.format[k] = 7 if k == 0 else 1
            t_full = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                _, df2, _ = ctx.encode(tfull, dfull, fmt=gsbc.FMT_BANDS, blocks=blocks)
                e1.record(stream)
                torch.cuda.synchronize()
                t_full.append(e0.elapsed_time(e1))
            # the degree-1 class in per-band streams (Fig. SetupD) and in Fig.
            # SetupC (four primitives' bands 0..3 per block): PSNR of its
            # decoded texels and its bytes per primitive
            def class1_row(label, tex_c, d_c, fmts):
                d_c = d_c.copy()
                for k, f in enumerate(fmts):
                    d_c.format[k] = f
                b, d3, _ = ctx.encode(tex_c, d_c, fmt=gsbc.FMT_BANDS, blocks=blocks)
                dec = ctx.decode(b, d3)
                diff = dec[..., :3].to(torch.int32) - tex_c[..., :3].to(torch.int32)
                mse = float((diff * diff).sum(dtype=torch.float64).item()) / (d3.n_pad * 12)
                return {"layout": label, "psnr_db": round(float(10 * np.log10(255.0 ** 2 / mse)), 2),
                        "bytes_per_primitive": round(d3.payload_bytes / counts[1], 3)}

            deg1 = None
            if counts[1]:
                _, _, texq, descq = ctx.reorder_degrees(posg_d, shg_d,
                                                        params=gsbc.default_params(arrangement=gsbc.ARR_QUAD))
                deg1 = [class1_row("SetupD: 4 BC1", texg[1], descg[1], [1] * 4),
                        class1_row("SetupC: BC1", texq[1], descq[1], [1]),
                        class1_row("SetupD: BC7 + 3 BC1", texg[1], descg[1], [7, 1, 1, 1]),
                        class1_row("SetupD: 4 BC7", texg[1], descg[1], [7] * 4),
                        class1_row("SetupC: BC7", texq[1], descq[1], [7])]
                del texq
            degrees = {"workload": f"{n:,} primitives, SH degree 0..3 drawn with probabilities {list(mix)}, "
                                   "band 0 BC7 + the other kept bands BC1, classes in one batch",
                       "degree1_layouts": deg1,
                       "class_counts": counts, "reorder_ms": round(float(np.median(t_re)), 3),
                       "encode_classes_ms": round(float(np.median(t_cls)), 3),
                       "encode_all_bands_ms": round(float(np.median(t_full)), 3),
                       "bytes_per_primitive_classes": round(bytes_cls / n, 3),
                       "bytes_per_primitive_all_bands": round(df2.payload_bytes / n, 3)}
            del posg_d, shg_d, permg, texg, tx, bufs, tfull
            torch.cuda.empty_cache()

        progress("arrangements and degree classes done")
        # ---- decode_eval on the 3,145,728-primitive scene at 1,024 directions
        roof_de = None
        if not args.no_large:
            del out
            torch.cuda.empty_cache()
            c3 = synth.CONFIGS["large"]
            pos3, sh3 = synth.make_scene(c3["n"], c3["clusters"], c3["comps"], c3["seed"])
            dirs3 = torch.from_numpy(synth.make_dirs(c3["dirs"], seed=c3["seed"])).to(dev)
            pos3_d, sh3_d = torch.from_numpy(pos3).to(dev), torch.from_numpy(sh3).to(dev)
            p3, t3, dd = ctx.reorder(pos3_d, sh3_d)
            b3, dd2, _ = ctx.encode(t3, dd, fmt=gsbc.FMT_AUTO, rate=c3["rate"])
            # timed reorder and rate-controlled encode of this scene (both
            # formats on every band, then the exact 6 bits/texel choice)
            t_re, t_en = [], []
            for i in range(3):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                e0.record(stream)
                p3, t3, dd = ctx.reorder(pos3_d, sh3_d, out=(p3, t3))
                e1.record(stream)
                b3, dd2, _ = ctx.encode(t3, dd, fmt=gsbc.FMT_AUTO, rate=c3["rate"], blocks=b3)
                e2.record(stream)
                torch.cuda.synchronize()
                t_re.append(e0.elapsed_time(e1) * 1e-3)
                t_en.append(e1.elapsed_time(e2) * 1e-3)
            # the reorder's device time: the same call with no desc only
            # enqueues (no read-back of the ranges, no wait); four calls back
            # to back between the events, so each call's host work overlaps
            # the previous call's kernels and the events bracket device time
            t_rd = []
            for i in range(5):
                e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
                e0.record(stream)
                for _ in range(4):
                    ctx.reorder(pos3_d, sh3_d, out=(p3, t3), want_desc=False)
                e1.record(stream)
                torch.cuda.synchronize()
                t_rd.append(e0.elapsed_time(e1) * 1e-3 / 4)
            nblk3 = dd.blocks_per_stream
            budget = int(c3["rate"] * 16 * 16 * nblk3 // 8)       # bits per texel x texels, in bytes
            # reorder bytes per primitive: range pass (SH 192 + position 12
            # read, band-0 colour 12 written), key pass (position 12 + colour
            # 12 read, key word 8 written), four sort passes of 8-9 bit digits
            # over key words that carry the index (word 8 read, 8 written;
            # then twice the tile counts' read 8 + 8 read + 8 written; then
            # 8 + 8 read and the index 4 written), gather (perm 4 + SH 192
            # read, texels 64 written)
            re_bytes_per_prim = 216 + 32 + (16 + 24 + 24 + 20) + 260
            re_s = float(np.median(t_re))
            large_enc = {"workload": "3,145,728 primitives (256 clusters, 256-component DC mixture, seed 3), "
                                     "6 bits/texel: band 0 BC7, 7 of bands 1..15 BC7, the rest BC1",
                         "reorder_ms": round(re_s * 1e3, 3), "reorder_ms_min": round(float(np.min(t_re)) * 1e3, 3),
                         "reorder_gb_s": round(re_bytes_per_prim * c3["n"] / re_s / 1e9, 1),
                         "reorder_hbm_frac": round(re_bytes_per_prim * c3["n"] / re_s / HBM_PEAK, 4),
                         "reorder_device_ms": round(float(np.median(t_rd)) * 1e3, 3),
                         "reorder_device_ms_min": round(float(np.min(t_rd)) * 1e3, 3),
                         "reorder_device_hbm_frac": round(re_bytes_per_prim * c3["n"] / float(np.median(t_rd)) / HBM_PEAK, 4),
                         "encode_ms": round(float(np.median(t_en)) * 1e3, 3),
                         "encode_ms_min": round(float(np.min(t_en)) * 1e3, 3),
                         "blocks_coded": 2 * 16 * nblk3,
                         "encode_mblocks_s": round(2 * 16 * nblk3 / float(np.median(t_en)) / 1e6, 2),
                         "payload_bytes": int(dd2.payload_bytes), "budget_bytes": budget,
                         "rate_exact": int(dd2.payload_bytes) == budget,
                         "bc7_bands": int((dd2.formats() == gsbc.FMT_BC7).sum())}
            del t3, sh3_d
            out3 = torch.empty((c3["dirs"], c3["n"], 3), dtype=torch.float32, device=dev)
            ctx.decode_eval(b3, dd2, dirs3, out=out3)
            torch.cuda.synchronize()
            t_de = kernel_ms(ctx, "decode_eval", lambda: ctx.decode_eval(b3, dd2, dirs3, out=out3), 5)
            de_s = float(np.mean(t_de)) * 1e-3
            # the same kernel at half the directions: T(V) = P + V s splits a
            # launch into the part that does not grow with the directions
            # (each workgroup's decode prologue, launch and tail) and the
            # per-direction evaluation and stores
            half = c3["dirs"] // 2
            t_half = kernel_ms(ctx, "decode_eval", lambda: ctx.decode_eval(b3, dd2, dirs3[:half], out=out3[:half]), 5)
            th, tf_ = float(np.median(t_half)), float(np.median(t_de))
            split = {"dirs": [half, c3["dirs"]], "ms": [round(th, 4), round(tf_, 4)],
                     "fixed_ms": round(2 * th - tf_, 4), "per_direction_us": round((tf_ - th) / half * 1e3, 4)}
            # every primitive's colour from one view position (its own direction)
            pos3d = torch.from_numpy(pos3).to(dev)
            view = (0.5, 0.5, 2.5)
            ctx.decode_eval_view(b3, dd2, pos3d, p3, view)
            t_view = kernel_ms(ctx, "decode_eval_view", lambda: ctx.decode_eval_view(b3, dd2, pos3d, p3, view), 3)
            view_s = float(np.median(t_view)) * 1e-3
            view_leg = {"workload": "3,145,728 primitives, one view position, each primitive at its own direction",
                        "ms": med_min(t_view), "gslots_s": round(c3["n"] / view_s / 1e9, 3),
                        "bytes": int(dd2.payload_bytes + c3["n"] * (12 + 4 + 12))}
            view_leg["gb_s"] = round(view_leg["bytes"] / view_s / 1e9, 1)
            # the fused colour stage: a 1920 x 1088 image of 16 x 16 tiles whose
            # front-to-back lists come from projecting the scene from the same
            # view position (footprints 0.7-6 px); every entry's colour decoded
            # in the tile's workgroup, nothing per primitive written to memory
            mu3 = synth.make_opacity(c3["n"], seed=c3["seed"])
            foot3, ts3, lst3 = synth.make_tiles(pos3, view, 120, 68, seed=c3["seed"], sigma=(0.7, 6.0))
            slot3 = np.argsort(p3.cpu().numpy().view(np.uint32)).astype(np.int32)
            mu3d, foot3d = torch.from_numpy(mu3).to(dev), torch.from_numpy(foot3).to(dev)
            ts3d = torch.from_numpy(ts3.astype(np.int32)).to(dev)
            lst3d = torch.from_numpy(slot3[lst3]).to(dev)
            img3, tr3 = ctx.blend_tiles(b3, dd2, pos3d, p3, view, mu3d, foot3d, ts3d, lst3d, 120, 68)
            t_bl = kernel_ms(ctx, ("tile_order", "blend_tiles"), lambda: ctx.blend_tiles(b3, dd2, pos3d, p3, view, mu3d, foot3d, ts3d,
                                                                         lst3d, 120, 68, image=img3,
                                                                         transmittance=tr3), 3)
            bl_s = float(np.median(t_bl)) * 1e-3
            entries = int(ts3[-1])
            colour_leg = {"workload": "1920x1088 image (120x68 tiles of 16x16), 3,145,728 primitives projected from "
                                      "the view position, footprint sigmas 0.7-6 px, front-to-back tile lists",
                          "ms": med_min(t_bl), "list_entries": entries,
                          "max_entries_per_tile": int(np.diff(ts3.astype(np.int64)).max()),
                          "gentries_s": round(entries / bl_s / 1e9, 3),
                          "listed_pixel_pairs_gs": round(256 * entries / bl_s / 1e9, 1),
                          # 18 issue slots per pixel-entry pair at least (footprint 7, exp 4,
                          # weights and transmittance 4, colour 3); tiles stop at T = 0 exactly,
                          # so this counts listed pairs, not executed ones
                          "alu_frac_listed_pairs": round(18 * 256 * entries / bl_s / VALU_PEAK, 4)}
            # the two-pass form: every primitive's colour decoded once (the
            # view decode), then the blend reads those colours (bit-identical)
            cols3 = ctx.decode_eval_view(b3, dd2, pos3d, p3, view)
            ctx.blend_tiles_colours(cols3, p3, mu3d, foot3d, ts3d, lst3d, 120, 68, image=img3, transmittance=tr3)
            t_bl2 = kernel_ms(ctx, ("decode_eval_view", "tile_order", "blend_tiles"),
                              lambda: (ctx.decode_eval_view(b3, dd2, pos3d, p3, view, out=cols3),
                                       ctx.blend_tiles_colours(cols3, p3, mu3d, foot3d, ts3d, lst3d, 120, 68,
                                                               image=img3, transmittance=tr3)), 3)
            colour_leg["two_pass"] = {"ms": med_min(t_bl2), "view_decode_included": True,
                                      "gentries_s": round(entries / (float(np.median(t_bl2)) * 1e-3) / 1e9, 3)}
            del pos3d, p3, img3, tr3, lst3d, ts3d, foot3d, mu3d, cols3
            # context: a plain device fill of the same output (write ceiling)
            tf = []
            for i in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                out3.fill_(0.0)
                e1.record(stream)
                torch.cuda.synchronize()
                tf.append(e0.elapsed_time(e1) * 1e-3)
            fill_gbps = out3.numel() * 4 / float(np.median(tf)) / 1e9
            de_bytes = c3["dirs"] * c3["n"] * 12 + dd2.payload_bytes + c3["dirs"] * 12
            tr_de = traffic_bytes("k_decode_eval")
            roof_de = {"kernel": "k_decode_eval", "bound": "hbm", "achieved": de_bytes / de_s / 1e9,
                       "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": de_bytes / de_s / HBM_PEAK,
                       "traffic": tr_de, "launch_ms": de_s * 1e3, "launch_ms_stats": med_min(t_de),
                       "workload": "3,145,728 primitives x 1,024 directions, 6 bits/texel",
                       "split": split, "plain_fill_gbps": round(fill_gbps, 1),
                       "fill_ms": med_min(tf, 1e3), "view": view_leg, "colour_stage": colour_leg,
                       "encode": large_enc}
            del out3, b3, pos3_d
            torch.cuda.empty_cache()
        progress("large scene legs done")
        batch = None if args.no_batch else batch_leg(ctx, stream, dev, args.batch_scenes, max(3, args.steps))
        ctx.close()
    progress("batch leg done")
    served = None if args.no_serve else serve_leg(dev, args.serve_requests)
    progress("serving leg done")

    cpu = None if args.no_cpu else cpu_baseline(pos, sh, dirs, rate)
    line = {
        "metric": "Mblocks/s BC7 & BC1 encode; decode+SH-eval GB/s; p50/p99 served latency",
        "value": round(value, 3), "unit": "Mblocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "1,048,576 primitives (32 clusters, 64-component DC mixture, seed 2): "
                               "reorder + BC1 and BC7 encode of all 16 bands + 6 bits/texel band choice "
                               "+ decode_eval at 64 directions",
                   "n_prims": n, "blocks_per_format": 16 * nblk, "rate_bits_per_texel": rate, "dirs": V},
        "stages_ms": {"reorder": med_min(stage[:, 0], 1.0, 3),
                      "encode_auto": med_min(stage[:, 1], 1.0, 3),
                      "decode_eval": med_min(stage[:, 2], 1.0, 3),
                      "step": med_min(stage.sum(axis=1), 1.0, 3)},
        "bc7_encode_mblocks_s": round(rates["bc7"], 3),
        "bc1_encode_mblocks_s": round(rates["bc1"], 3),
        "format_encode_ms": {"bc7": rates["bc7_ms"], "bc1": rates["bc1_ms"]},
        "psnr_db_per_band": psnr,
        "arrangements": arrangements,
        "degree_classes": degrees,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "roofline": roof,
        "valu_issue": valu or None,
        "roofline_decode_eval": roof_de,
        "batch": batch,
        "serving": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def batch_leg(ctx, stream, dev, n_scenes, reps):
    """64 scenes of log-uniform size in [5e4, 2e6] primitives (seed 4; scene i
    drawn with seed 1000 + i on the device), band 0 BC7 and bands 1..15 BC1:
    one autotuned, graph-captured batched call against 64 single-scene calls.
    Both must give identical bitstreams."""
    import torch
    from paper_2607_14513_amd import autotune, gsbc, synth
    sizes = synth.batch_sizes(n_scenes, seed=4)
    texs, descs = [], []
    for i, n in enumerate(sizes):
        pos_i, sh_i = synth.make_scene_device(n, seed=1000 + i, device=dev)
        _, tex_i, d_i = ctx.reorder(pos_i, sh_i)
        for k in range(16):
            d_i.format[k] = gsbc.FMT_BC7 if k == 0 else gsbc.FMT_BC1
        texs.append(tex_i)
        descs.append(d_i)
        del pos_i, sh_i
    torch.cuda.synchronize()
    nblocks = sum(16 * d.blocks_per_stream for d in descs)
    pay = [d.blocks_per_stream * (16 + 15 * 8) + 16 * 16 for d in descs]
    plain_out = [torch.empty(p, dtype=torch.uint8, device=dev) for p in pay]
    batch_out = [torch.empty(p, dtype=torch.uint8, device=dev) for p in pay]

    def plain_pass():
        outs = []
        for i in range(n_scenes):
            _, di, _ = ctx.encode(texs[i], descs[i], fmt=gsbc.FMT_BANDS, blocks=plain_out[i])
            outs.append(di)
        return outs

    plain_pass()
    torch.cuda.synchronize()
    t_plain = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pd = plain_pass()
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
    tuning, tinfo = autotune.tune(ctx, texs, descs, batch_out, repeats=2,
                                  log=lambda m: print(m, file=sys.stderr, flush=True))
    bd, _ = ctx.encode_batch(texs, descs, batch_out, tuning=tuning)    # capture (or replay)
    torch.cuda.synchronize()
    t_batch, t_dev = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        bd, _ = ctx.encode_batch(texs, descs, batch_out, tuning=tuning)
        e1.record(stream)
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t0)
        t_dev.append(e0.elapsed_time(e1) * 1e-3)
    same = all(pd[i].payload_bytes == bd[i].payload_bytes and
               torch.equal(plain_out[i][:pd[i].payload_bytes], batch_out[i][:bd[i].payload_bytes])
               for i in range(n_scenes))
    tp, tb = float(np.median(t_plain)), float(np.median(t_batch))
    return {"workload": f"{n_scenes} scenes, {sum(sizes)} primitives (log-uniform 5e4..2e6, seed 4), "
                        "band 0 BC7 + bands 1..15 BC1",
            "blocks": int(nblocks), "plain_ms": round(tp * 1e3, 3), "batched_ms": round(tb * 1e3, 3),
            "batched_device_ms": round(float(np.median(t_dev)) * 1e3, 3),
            "plain_mblocks_s": round(nblocks / tp / 1e6, 3), "batched_mblocks_s": round(nblocks / tb / 1e6, 3),
            "speedup": round(tp / tb, 3), "identical_bitstreams": bool(same),
            "tuning": tuning.as_dict(), "autotune": {k: tinfo[k] for k in ("ms", "default_ms", "configs_timed",
                                                                          "search_s", "cached") if k in tinfo}}


def serve_leg(dev, count, slots=4):
    """Poisson arrivals of encode (70%) and decode_eval (30%) requests; N
    log-uniform in [1e4, 4e6] primitives (slices of a 4M-primitive scene drawn
    on the device, seed 5), V log-uniform in [1, 1024], each decode reading
    the scene of an earlier encode; encodes at 6 bits per texel stay
    resident; 200 GB HBM budget.  The arrival rate is 70% of the plain path's
    capacity, measured first by serving a calibration set one request at a
    time.  The same arrivals are then served twice: by `slots` overlapping
    slots (continuous batching) and by the plain path (one slot, first come
    first served).  Sampled results are digested in both runs and re-run
    alone; all three must agree."""
    import torch
    from paper_2607_14513_amd import serve, synth
    pool_n = 4_000_000
    pos, sh = synth.make_scene_device(pool_n, seed=5, device=dev)
    torch.cuda.synchronize()
    # plain capacity: one slot, requests back to back
    cal = serve.make_requests(60, 1e9, seed=55, pool_n=pool_n)
    s1 = serve.Server(pos, sh, slots=1, hbm_budget=200e9, digest_ids=set())
    try:
        s1.run(cal[:6])                       # warm-up (contexts, allocator)
        t0 = time.perf_counter()
        s1.run(cal[6:])
        service = (time.perf_counter() - t0) / len(cal[6:])
    finally:
        s1.close()
    del s1
    torch.cuda.empty_cache()
    capacity = 1.0 / service
    lam = 0.7 * capacity
    sample = set(range(0, count, max(1, count // 24)))
    out = {"workload": f"{count} requests, Poisson arrivals at {lam:.2f}/s (70% of the measured one-at-a-time "
                       f"capacity {capacity:.2f}/s), 70% encode at 6 bits/texel / 30% decode_eval of an earlier "
                       "request's scene, N log-uniform 1e4..4e6, V log-uniform 1..1024, 200 GB budget",
           "arrival_rate_hz": round(lam, 3), "plain_capacity_hz": round(capacity, 3)}
    digests = {}
    for label, nslots in (("served", slots), ("plain", 1)):
        reqs = serve.make_requests(count, lam, seed=5, pool_n=pool_n)
        srv = serve.Server(pos, sh, slots=nslots, hbm_budget=200e9, digest_ids=sample)
        try:
            done = srv.run(reqs)
            summ = serve.summarize(done, srv.t_elapsed, srv.t0)
            summ.update({"slots": nslots, "evicted_scenes": srv.evicted, "arena_growths": srv.arena_growths()})
            digests[label] = {r.rid: r.digest for r in done if r.rid in sample and r.error is None}
            if label == "served":
                same = checked = 0
                for r in sorted(done, key=lambda r: r.rid):
                    if r.rid in sample and r.error is None:
                        checked += 1
                        same += int(srv.run_alone(r)[0] == r.digest)
                summ.update({"identity_checked": checked, "identity_same_alone": same})
        finally:
            srv.close()
        del srv
        torch.cuda.empty_cache()
        out[label] = summ
    common = set(digests["served"]) & set(digests["plain"])
    out["identity_same_plain"] = sum(int(digests["served"][k] == digests["plain"][k]) for k in common)
    out["identity_checked_plain"] = len(common)
    return out


def cpu_baseline(pos, sh, dirs, rate):
    """The oracle, untuned, on a bounded sample of the step: full reorder, BC1
    and BC7 on 8,192 sampled blocks each, decode_eval of 16,384 slots at all
    directions; scaled to the whole step's Mblocks/s."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)
    n = pos.shape[0]
    nblk = (n + 15) // 16
    t = time.perf_counter()
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    t_reorder = time.perf_counter() - t
    rng = np.random.default_rng(0)
    S = 8192
    bands = rng.integers(0, 16, S)
    blks = rng.integers(0, nblk, S)
    sample = tex[bands, blks]
    O._load().ref_init()
    t = time.perf_counter()
    O.bc1_encode(sample)
    t_bc1 = (time.perf_counter() - t) / S
    t = time.perf_counter()
    O.bc7_encode(sample)
    t_bc7 = (time.perf_counter() - t) / S
    fmt = np.array([7] + [1] * 15, np.uint8)
    slots = np.sort(rng.choice(n, 16384, replace=False)).astype(np.uint32)
    blk_ids = np.unique(slots // 16)
    mini = tex[:, blk_ids]
    payload, off, _ = O.encode(mini, fmt)
    where = {int(b): i for i, b in enumerate(blk_ids)}
    renum = np.array([16 * where[int(s) // 16] + int(s) % 16 for s in slots], np.uint32)
    t = time.perf_counter()
    O.decode_eval(payload, off, fmt, vmin, vmax, dirs, renum, with_scale=False)
    t_de = (time.perf_counter() - t) / len(slots)
    step = t_reorder + 16 * nblk * (t_bc1 + t_bc7) + n * t_de
    # the same oracle on one thread, on a smaller sample (the reorder is
    # single-threaded either way, so its full-scene time is reused)
    O.set_threads(1)
    S1 = 256
    t = time.perf_counter()
    O.bc1_encode(sample[:S1])
    t1_bc1 = (time.perf_counter() - t) / S1
    t = time.perf_counter()
    O.bc7_encode(sample[:S1])
    t1_bc7 = (time.perf_counter() - t) / S1
    t = time.perf_counter()
    O.decode_eval(payload, off, fmt, vmin, vmax, dirs, renum[:2048], with_scale=False)
    t1_de = (time.perf_counter() - t) / 2048
    O.set_threads(threads)
    step1 = t_reorder + 16 * nblk * (t1_bc1 + t1_bc7) + n * t1_de
    return {"value": round(2 * 16 * nblk / step / 1e6, 6), "unit": "Mblocks/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"full reorder of {n} primitives ({t_reorder:.2f} s); BC1 and BC7 on {S} sampled "
                      f"blocks ({t_bc1 * 1e3:.3f} / {t_bc7 * 1e3:.3f} ms per block); decode_eval of "
                      f"{len(slots)} slots x {len(dirs)} directions; scaled to one step of "
                      f"{2 * 16 * nblk} blocks ({step:.1f} s)",
            "single_thread": {
                "value": round(2 * 16 * nblk / step1 / 1e6, 6), "unit": "Mblocks/s", "cores": 1,
                "sample": f"BC1 and BC7 on {S1} of the sampled blocks ({t1_bc1 * 1e3:.3f} / {t1_bc7 * 1e3:.3f} "
                          f"ms per block); decode_eval of 2048 slots x {len(dirs)} directions; the reorder "
                          f"time above; scaled to one step ({step1:.1f} s)"}}


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), else the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


if __name__ == "__main__":
    main()
