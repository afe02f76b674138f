// api.cpp -- the C ABI (include/gsbc.h): argument checks, scratch arena,
// stream, error reporting, and the order in which each call's kernels are
// enqueued.  All computation happens in the kernels.
#include "../../include/gsbc.h"
#include "gsbc_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <vector>

using namespace gsbc;


struct gsbc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *arena = nullptr;          // grows on demand; freed with the context
    size_t arena_bytes = 0;
    void *small = nullptr;          // fixed device block: range, selection, SSE sums, offsets
    void *pinned = nullptr;         // host staging for read-backs
    char err[512] = {0};
    // kernel timing (gsbc_profile_enable)
    bool profiling = false;
    struct Rec { const char *name; size_t ev; };
    std::vector<hipEvent_t> events;  // pairs: 2k start, 2k+1 end
    std::vector<Rec> recs;
};

namespace {

// The context whose call is running on this thread (for the timing hooks).
thread_local gsbc_ctx *t_active = nullptr;

struct ActiveGuard {
    explicit ActiveGuard(gsbc_ctx *c) { t_active = c; }
    ~ActiveGuard() { t_active = nullptr; }
};

// Device "small" block layout
constexpr size_t kRangeOff = 0;                  // RangeRec
constexpr size_t kSelOff = 512;                  // RateSel
constexpr size_t kSse1Off = 1024;                // 16 x u64
constexpr size_t kSse7Off = 1152;                // 16 x u64
constexpr size_t kOff1Off = 1280;                // 16 x u64
constexpr size_t kOff7Off = 1408;                // 16 x u64
constexpr size_t kSmallBytes = 2048;

std::atomic<long> g_alloc_count{0};

// Failure injection for tests: GSBC_FAULT=alloc:<k> makes the k-th scratch
// allocation of the process fail.
bool injected_alloc_failure()
{
    long k = g_alloc_count.fetch_add(1) + 1;
    const char *f = getenv("GSBC_FAULT");
    if (!f || strncmp(f, "alloc:", 6) != 0) return false;
    return atol(f + 6) == k;
}

gsbc_status fail(gsbc_ctx *ctx, gsbc_status code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

gsbc_status hip_fail(gsbc_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, GSBC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                                   \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, (what));  \
    } while (0)

gsbc_status begin(gsbc_ctx *ctx)
{
    if (!ctx) return GSBC_E_ARG;
    ctx->err[0] = 0;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    // a fault from earlier asynchronous work surfaces here
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "earlier work");
    return GSBC_OK;
}

gsbc_status ensure_arena(gsbc_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->arena_bytes) return GSBC_OK;
    if (ctx->arena) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        HIP_TRY(ctx, hipFree(ctx->arena), "hipFree");
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
    }
    if (injected_alloc_failure()) return fail(ctx, GSBC_E_NOMEM, "scratch allocation of %zu bytes failed (injected)", bytes);
    size_t want = (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
    hipError_t e = hipMalloc(&ctx->arena, want);
    if (e != hipSuccess) {
        ctx->arena = nullptr;
        (void)hipGetLastError();
        return fail(ctx, GSBC_E_NOMEM, "scratch allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    ctx->arena_bytes = want;
    return GSBC_OK;
}

uint64_t pad16(uint64_t n) { return (n + 15) / 16 * 16; }
uint64_t align16(uint64_t x) { return (x + 15) & ~(uint64_t)15; }

gsbc_params resolve(const gsbc_params *p)
{
    gsbc_params d;
    gsbc_default_params(&d);
    return p ? *p : d;
}

gsbc_status check_params(gsbc_ctx *ctx, const gsbc_params &p)
{
    if (p.grid_bits > 10) return fail(ctx, GSBC_E_ARG, "grid_bits %u > 10", p.grid_bits);
    if (p.refine_steps > 8) return fail(ctx, GSBC_E_ARG, "refine_steps %u > 8", p.refine_steps);
    if (p.bc7_mode_mask == 0 || p.bc7_mode_mask > 0xFF) return fail(ctx, GSBC_E_ARG, "bc7_mode_mask 0x%x not in 1..0xFF", p.bc7_mode_mask);
    return GSBC_OK;
}

gsbc_status check_desc(gsbc_ctx *ctx, const gsbc_stream_desc *d)
{
    if (!d) return fail(ctx, GSBC_E_ARG, "desc is NULL");
    if (d->n_prims == 0 || d->n_prims > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "desc.n_prims %llu out of range", (unsigned long long)d->n_prims);
    if (d->n_pad != pad16(d->n_prims) || d->blocks_per_band * 16 != d->n_pad)
        return fail(ctx, GSBC_E_ARG, "desc sizes inconsistent (n_prims %llu, n_pad %llu, blocks %llu)",
                    (unsigned long long)d->n_prims, (unsigned long long)d->n_pad, (unsigned long long)d->blocks_per_band);
    return GSBC_OK;
}

gsbc_status check_stream(gsbc_ctx *ctx, const gsbc_stream_desc *d)
{
    gsbc_status s = check_desc(ctx, d);
    if (s) return s;
    uint64_t pos = 0;
    for (int k = 0; k < 16; k++) {
        if (d->format[k] != GSBC_FMT_BC1 && d->format[k] != GSBC_FMT_BC7)
            return fail(ctx, GSBC_E_ARG, "desc.format[%d] = %u is not BC1 or BC7", k, d->format[k]);
        if (d->offset[k] != pos) return fail(ctx, GSBC_E_ARG, "desc.offset[%d] does not follow the stream layout", k);
        pos = align16(pos + d->blocks_per_band * (d->format[k] == GSBC_FMT_BC1 ? 8 : 16));
    }
    if (d->payload_bytes != pos) return fail(ctx, GSBC_E_ARG, "desc.payload_bytes inconsistent");
    return GSBC_OK;
}

BandArgs band_args(const gsbc_stream_desc *d)
{
    BandArgs b;
    for (int k = 0; k < 16; k++) {
        b.offset[k] = d->offset[k];
        b.format[k] = d->format[k];
        b.vmin[k] = d->vmin[k];
        b.delta[k] = (d->vmax[k] - d->vmin[k]) / 255.0f;
    }
    return b;
}

char *small_ptr(gsbc_ctx *ctx, size_t off) { return static_cast<char *>(ctx->small) + off; }

}  // namespace

namespace gsbc {

void trace_begin(const char *kernel, hipStream_t st)
{
    gsbc_ctx *c = t_active;
    if (!c || !c->profiling) return;
    size_t k = c->recs.size();
    while (c->events.size() < 2 * (k + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->events.push_back(e);
    }
    c->recs.push_back({kernel, 2 * k});
    (void)hipEventRecord(c->events[2 * k], st);
}

void trace_end(hipStream_t st)
{
    gsbc_ctx *c = t_active;
    if (!c || !c->profiling || c->recs.empty()) return;
    (void)hipEventRecord(c->events[c->recs.back().ev + 1], st);
}

}  // namespace gsbc

extern "C" {

void gsbc_default_params(gsbc_params *p)
{
    if (!p) return;
    p->grid_bits = 3;
    p->refine_steps = 2;
    p->bc7_mode_mask = 0xFF;
}

gsbc_status gsbc_create(gsbc_ctx **out, int device, void *hip_stream)
{
    if (!out) return GSBC_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { (void)hipGetLastError(); return GSBC_E_DEVICE; }
    if (device < 0 || device >= ndev) return GSBC_E_ARG;
    gsbc_ctx *ctx = new gsbc_ctx();
    ctx->device = device;
    auto bail = [&](gsbc_status s) {
        if (ctx->small) (void)hipFree(ctx->small);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return s;
    };
    if (hipSetDevice(device) != hipSuccess) return bail(GSBC_E_DEVICE);
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        // a blocking stream: ordered with work on the legacy null stream
        if (hipStreamCreate(&ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
        ctx->own_stream = true;
    }
    if (hipMalloc(&ctx->small, kSmallBytes) != hipSuccess) return bail(GSBC_E_NOMEM);
    if (hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault) != hipSuccess) return bail(GSBC_E_NOMEM);
    if (upload_bc1_tables(ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
    if (upload_bc7_tables(device, ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
    *out = ctx;
    return GSBC_OK;
}

gsbc_status gsbc_destroy(gsbc_ctx *ctx)
{
    if (!ctx) return GSBC_E_ARG;
    gsbc_status s = GSBC_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) s = GSBC_E_DEVICE;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) s = GSBC_E_DEVICE;
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->small) (void)hipFree(ctx->small);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return s;
}

const char *gsbc_last_error(const gsbc_ctx *ctx) { return ctx ? ctx->err : "no context"; }

gsbc_status gsbc_sync(gsbc_ctx *ctx)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return GSBC_OK;
}

gsbc_status gsbc_query_sizes(uint64_t n, uint32_t n_dirs, uint64_t *textures_bytes, uint64_t *max_blocks_bytes,
                             uint64_t *out_bytes)
{
    if (n == 0 || n > 0x7FFFFFFFull) return GSBC_E_ARG;
    uint64_t np = pad16(n);
    if (textures_bytes) *textures_bytes = 16 * np * 4;
    if (max_blocks_bytes) *max_blocks_bytes = 16 * (np / 16) * 16;
    if (out_bytes) *out_bytes = (uint64_t)n_dirs * n * 12;
    return GSBC_OK;
}

gsbc_status gsbc_reorder(gsbc_ctx *ctx, const float *pos, const float *sh, uint64_t n, const gsbc_params *params,
                         uint32_t *perm, uint8_t *textures, gsbc_stream_desc *desc)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!pos || !sh || !perm || !textures || !desc) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (n == 0 || n > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "n = %llu not in 1..2^31-1", (unsigned long long)n);
    if ((reinterpret_cast<uintptr_t>(sh) & 15) || (reinterpret_cast<uintptr_t>(textures) & 15) ||
        (reinterpret_cast<uintptr_t>(pos) & 3) || (reinterpret_cast<uintptr_t>(perm) & 3))
        return fail(ctx, GSBC_E_ARG, "sh and textures must be 16-byte aligned, pos and perm 4-byte aligned");
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    if ((s = ensure_arena(ctx, reorder_scratch_bytes(n, p.grid_bits)))) return s;
    RangeRec *range = reinterpret_cast<RangeRec *>(small_ptr(ctx, kRangeOff));
    HIP_TRY(ctx, launch_reorder(pos, sh, n, p.grid_bits, perm, textures, ctx->arena, range, ctx->stream), "reorder launch");
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, range, sizeof(RangeRec), hipMemcpyDeviceToHost, ctx->stream), "range read-back");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "reorder");
    const RangeRec *r = static_cast<const RangeRec *>(ctx->pinned);
    memset(desc, 0, sizeof *desc);
    for (int k = 0; k < 16; k++) { desc->vmin[k] = r->vmin[k]; desc->vmax[k] = r->vmax[k]; }
    desc->n_prims = n;
    desc->n_pad = pad16(n);
    desc->blocks_per_band = desc->n_pad / 16;
    return GSBC_OK;
}

gsbc_status gsbc_encode(gsbc_ctx *ctx, const uint8_t *textures, gsbc_stream_desc *desc, int format, double rate,
                        const gsbc_params *params, uint8_t *blocks, uint64_t blocks_capacity, int64_t *band_sse)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!textures || !blocks) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(textures) & 15) || (reinterpret_cast<uintptr_t>(blocks) & 15))
        return fail(ctx, GSBC_E_ARG, "textures and blocks must be 16-byte aligned");
    if ((s = check_desc(ctx, desc))) return s;
    if (format != GSBC_FMT_AUTO && format != GSBC_FMT_BC1 && format != GSBC_FMT_BC7)
        return fail(ctx, GSBC_E_ARG, "format %d is not AUTO(0), BC1(1) or BC7(7)", format);
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    const uint64_t nblk = desc->blocks_per_band;
    unsigned long long *sse1 = reinterpret_cast<unsigned long long *>(small_ptr(ctx, kSse1Off));
    unsigned long long *sse7 = reinterpret_cast<unsigned long long *>(small_ptr(ctx, kSse7Off));

    EncodeArgs a;
    memset(&a, 0, sizeof a);
    a.textures = textures;
    a.nblk = nblk;
    a.refine_steps = p.refine_steps;
    a.mode_mask = p.bc7_mode_mask;

    uint64_t host_off[16];
    uint32_t host_fmt[16];
    uint64_t payload = 0;
    if (format != GSBC_FMT_AUTO) {
        for (int k = 0; k < 16; k++) {
            host_off[k] = payload;
            host_fmt[k] = (uint32_t)format;
            payload = align16(payload + nblk * (format == GSBC_FMT_BC1 ? 8 : 16));
        }
        if (blocks_capacity < payload)
            return fail(ctx, GSBC_E_BUFFER, "blocks_capacity %llu < payload %llu bytes", (unsigned long long)blocks_capacity,
                        (unsigned long long)payload);
        if ((s = ensure_arena(ctx, bc7_scratch_bytes(16 * nblk)))) return s;
        a.keys = static_cast<uint32_t *>(ctx->arena);
        HIP_TRY(ctx, launch_fill_u64(sse1, 32, 0, ctx->stream), "clear");
        a.band0 = 0;
        a.nbands = 16;
        a.out = blocks;
        memcpy(a.out_offset, host_off, sizeof host_off);
        a.band_sse = format == GSBC_FMT_BC1 ? sse1 : sse7;
        HIP_TRY(ctx, format == GSBC_FMT_BC1 ? launch_bc1_encode(a, ctx->stream) : launch_bc7_encode(a, ctx->stream), "encode launch");
    } else {
        double kd = 4.0 * rate - 17.0;
        if (!(kd >= 0.0 && kd <= 15.0) || kd != floor(kd))
            return fail(ctx, GSBC_E_INFEASIBLE, "rate %.17g bits/texel needs 4*rate-17 BC7 bands, not an integer in 0..15", rate);
        const uint32_t k = (uint32_t)kd;
        payload = (uint64_t)(k + 1) * 16 * nblk + (uint64_t)(15 - k) * align16(8 * nblk);
        if (blocks_capacity < payload)
            return fail(ctx, GSBC_E_BUFFER, "blocks_capacity %llu < payload %llu bytes", (unsigned long long)blocks_capacity,
                        (unsigned long long)payload);
        const uint64_t s1 = align16(8 * nblk), s7 = 16 * nblk;
        if ((s = ensure_arena(ctx, 16 * s1 + 16 * s7 + bc7_scratch_bytes(16 * nblk)))) return s;
        uint8_t *buf1 = static_cast<uint8_t *>(ctx->arena), *buf7 = buf1 + 16 * s1;
        a.keys = reinterpret_cast<uint32_t *>(buf7 + 16 * s7);
        uint64_t off1[16], off7[16];
        for (int q = 0; q < 16; q++) { off1[q] = q * s1; off7[q] = q * s7; }
        uint64_t *doff1 = reinterpret_cast<uint64_t *>(small_ptr(ctx, kOff1Off));
        uint64_t *doff7 = reinterpret_cast<uint64_t *>(small_ptr(ctx, kOff7Off));
        uint64_t *stage = static_cast<uint64_t *>(ctx->pinned);
        memcpy(stage, off1, sizeof off1);
        memcpy(stage + 16, off7, sizeof off7);
        HIP_TRY(ctx, hipMemcpyAsync(doff1, stage, 2 * sizeof off1, hipMemcpyHostToDevice, ctx->stream), "offsets");
        HIP_TRY(ctx, launch_fill_u64(sse1, 32, 0, ctx->stream), "clear");
        a.out = buf7;
        memcpy(a.out_offset, off7, sizeof off7);
        a.band0 = 0;
        a.nbands = 16;
        a.band_sse = sse7;
        HIP_TRY(ctx, launch_bc7_encode(a, ctx->stream), "bc7 launch");
        a.out = buf1;
        memcpy(a.out_offset, off1, sizeof off1);
        a.band0 = 0;            // band 0 is always BC7; its BC1 SSE is reported too
        a.nbands = 16;
        a.band_sse = sse1;
        HIP_TRY(ctx, launch_bc1_encode(a, ctx->stream), "bc1 launch");
        RateSel *sel = reinterpret_cast<RateSel *>(small_ptr(ctx, kSelOff));
        HIP_TRY(ctx, launch_rate_select(sse1, sse7, band_args(desc), k, nblk, sel, ctx->stream), "rate select");
        HIP_TRY(ctx, launch_copy_streams(buf1, doff1, buf7, doff7, sel, nblk, blocks, ctx->stream), "stream copy");
        // stage[0..] is reused for the read-back below, after the H2D copy has run
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "encode");
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, sel, sizeof(RateSel), hipMemcpyDeviceToHost, ctx->stream), "selection read-back");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "encode");
        const RateSel *r = static_cast<const RateSel *>(ctx->pinned);
        for (int q = 0; q < 16; q++) { host_fmt[q] = r->format[q]; host_off[q] = r->offset[q]; }
        if (r->payload_bytes != payload) return fail(ctx, GSBC_E_DEVICE, "selected payload size disagrees with the budget");
    }
    char *stage = static_cast<char *>(ctx->pinned) + 1024;
    HIP_TRY(ctx, hipMemcpyAsync(stage, sse1, 32 * sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream), "sse read-back");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "encode");
    if (band_sse) {
        const uint64_t *h = reinterpret_cast<const uint64_t *>(stage);
        bool have1 = format != GSBC_FMT_BC7, have7 = format != GSBC_FMT_BC1;
        for (int q = 0; q < 16; q++) {
            band_sse[q] = have1 ? (int64_t)h[q] : -1;
            band_sse[16 + q] = have7 ? (int64_t)h[16 + q] : -1;
        }
    }
    for (int q = 0; q < 16; q++) { desc->format[q] = (uint8_t)host_fmt[q]; desc->offset[q] = host_off[q]; }
    desc->payload_bytes = payload;
    return GSBC_OK;
}

gsbc_status gsbc_decode(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc, uint8_t *textures_out)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!blocks || !textures_out) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(blocks) & 15) || (reinterpret_cast<uintptr_t>(textures_out) & 15))
        return fail(ctx, GSBC_E_ARG, "blocks and textures_out must be 16-byte aligned");
    if ((s = check_stream(ctx, desc))) return s;
    HIP_TRY(ctx, launch_decode(blocks, band_args(desc), desc->blocks_per_band, textures_out, ctx->stream), "decode launch");
    return GSBC_OK;
}

gsbc_status gsbc_decode_eval(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc, const float *dirs,
                             uint32_t n_dirs, const uint32_t *prim_idx, uint64_t m, float *out)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!blocks || !dirs || !out) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (reinterpret_cast<uintptr_t>(blocks) & 15) return fail(ctx, GSBC_E_ARG, "blocks must be 16-byte aligned");
    if ((reinterpret_cast<uintptr_t>(dirs) & 3) || (reinterpret_cast<uintptr_t>(out) & 3) ||
        (reinterpret_cast<uintptr_t>(prim_idx) & 3))
        return fail(ctx, GSBC_E_ARG, "dirs, prim_idx and out must be 4-byte aligned");
    if ((s = check_stream(ctx, desc))) return s;
    if (n_dirs == 0) return fail(ctx, GSBC_E_ARG, "n_dirs must be >= 1");
    if (m == 0) return fail(ctx, GSBC_E_ARG, "m must be >= 1");
    if (!prim_idx && m != desc->n_prims) return fail(ctx, GSBC_E_ARG, "prim_idx NULL requires m == n_prims");
    if (m > 0xFFFFFFFFull * 256) return fail(ctx, GSBC_E_ARG, "m too large");
    if ((s = ensure_arena(ctx, (size_t)n_dirs * 16 * sizeof(float)))) return s;
    HIP_TRY(ctx, launch_decode_eval(blocks, band_args(desc), desc->n_prims, dirs, n_dirs, prim_idx, m, out,
                                    static_cast<float *>(ctx->arena), ctx->stream), "decode_eval launch");
    return GSBC_OK;
}

gsbc_status gsbc_profile_enable(gsbc_ctx *ctx, int on)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ctx->profiling = on != 0;
    return GSBC_OK;
}

gsbc_status gsbc_profile_read(gsbc_ctx *ctx, uint32_t max_entries, char *names, uint32_t *counts, double *ms,
                              uint32_t *n_out)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    if (!n_out || (max_entries && (!names || !counts || !ms))) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    uint32_t n = 0;
    for (const gsbc_ctx::Rec &r : ctx->recs) {
        float t = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->events[r.ev], ctx->events[r.ev + 1]), "hipEventElapsedTime");
        uint32_t q = 0;
        while (q < n && strncmp(names + 64 * q, r.name, 63) != 0) q++;
        if (q == n) {
            if (n == max_entries) continue;
            snprintf(names + 64 * n, 64, "%s", r.name);
            counts[n] = 0;
            ms[n] = 0.0;
            n++;
        }
        counts[q]++;
        ms[q] += t;
    }
    ctx->recs.clear();
    *n_out = n;
    return GSBC_OK;
}

}  // extern "C"
