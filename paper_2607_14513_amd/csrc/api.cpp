// api.cpp -- the C ABI (include/gsbc.h): argument checks, scratch arena,
// stream, error reporting, and the order in which each call's kernels are
// enqueued.  All computation happens in the kernels.
#include "../../include/gsbc.h"
#include "gsbc_internal.h"

#include <cstddef>

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
    std::vector<void *> retired;    // arenas outgrown while kernels could still read them
    uint64_t arena_growths = 0;
    void *small = nullptr;          // fixed device block: range, selection, SSE sums, offsets
    void *pinned = nullptr;         // host staging for read-backs
    // the last gsbc_reorder (for gsbc_reorder_desc): its n and params
    bool reordered = false;
    uint64_t last_n = 0;
    gsbc_params last_p{};
    char err[512] = {0};
    // gsbc_encode_batch: the last plan (device tables + captured graph)
    hipStream_t side = nullptr;      // second stream for BC1 beside BC7
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<uint64_t> plan_sig;
    void *plan_mem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    unsigned long long *plan_sse = nullptr;
    bool capturing = false;
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
constexpr size_t kClassOff = 1536;               // 4 x u32 degree-class counts
constexpr size_t kSmallBytes = 2048;
static_assert(sizeof(gsbc::RangeRec) <= kSelOff, "RangeRec must fit before RateSel (and before the class counts read back beside it)");

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

// Grow the context's scratch arena to at least `bytes`.  The old arena may
// still be read by kernels queued on the stream, and freeing device memory
// waits for the whole device (other contexts' streams included), so it is
// retired, not freed: retired arenas are freed with the context.  Growth is
// at least twofold, so retired memory stays below the live arena's size.
// Calls within the sizes given to gsbc_reserve never grow it.
gsbc_status ensure_arena(gsbc_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->arena_bytes) return GSBC_OK;
    if (injected_alloc_failure()) return fail(ctx, GSBC_E_NOMEM, "scratch allocation of %zu bytes failed (injected)", bytes);
    size_t want = std::max(bytes, 2 * ctx->arena_bytes);
    want = (want + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, GSBC_E_NOMEM, "scratch allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    if (ctx->arena) ctx->retired.push_back(ctx->arena);
    ctx->arena = p;
    ctx->arena_bytes = want;
    ctx->arena_growths++;
    return GSBC_OK;
}

uint64_t pad16(uint64_t n) { return (n + 15) / 16 * 16; }
// Textures of the four degree classes: sum over L of (L+1)^2 streams of
// pad16(n_L) texels of 4 bytes, at most 4 (16 n + 15 (1 + 4 + 9 + 16))
// <= n_pad*64 + 1800 bytes.
uint64_t degree_textures_bytes(uint64_t n) { return pad16(n) * 64 + 1800; }
// Streams of an arrangement: one per band, one, or one per band group.
uint32_t streams_of(uint32_t arr) { return arr == GSBC_ARR_PRIM ? 1u : arr == GSBC_ARR_QUAD ? 4u : 16u; }
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
    if (p.order > 1) return fail(ctx, GSBC_E_ARG, "order %u is not 0 (sorted) or 1 (identity)", p.order);
    if (p.quantiser > 1) return fail(ctx, GSBC_E_ARG, "quantiser %u is not 0 (min/max) or 1 (99.5%% coverage)", p.quantiser);
    if (p.arrangement > GSBC_ARR_QUAD)
        return fail(ctx, GSBC_E_ARG, "arrangement %u is not BANDS(0), PRIM(1) or QUAD(2)", p.arrangement);
    return GSBC_OK;
}

// Bytes of one stream: a 0-bit stream (GSBC_FMT_NONE) stores no blocks.
uint64_t stream_bytes(uint32_t fmt, uint64_t nblk)
{
    return fmt == GSBC_FMT_NONE ? 0 : nblk * (fmt == GSBC_FMT_BC1 ? 8 : 16);
}

// A stream's format: BC1 or BC7; with the band arrangement also 0 bits.
bool stream_format_ok(uint32_t fmt, uint32_t arrangement)
{
    return fmt == GSBC_FMT_BC1 || fmt == GSBC_FMT_BC7 || (fmt == GSBC_FMT_NONE && arrangement == GSBC_ARR_BANDS);
}

gsbc_status check_desc(gsbc_ctx *ctx, const gsbc_stream_desc *d)
{
    if (!d) return fail(ctx, GSBC_E_ARG, "desc is NULL");
    if (d->n_prims == 0 || d->n_prims > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "desc.n_prims %llu out of range", (unsigned long long)d->n_prims);
    // the band arrangement may keep only the (L+1)^2 lowest bands (a degree
    // class), and the quad arrangement only its first stream (Fig. SetupC)
    const bool bands_ok = d->arrangement == GSBC_ARR_BANDS &&
                          (d->n_streams == 1 || d->n_streams == 4 || d->n_streams == 9 || d->n_streams == 16);
    const bool quad1_ok = d->arrangement == GSBC_ARR_QUAD && d->n_streams == 1;
    if (d->arrangement > GSBC_ARR_QUAD || (!bands_ok && !quad1_ok && d->n_streams != streams_of(d->arrangement)))
        return fail(ctx, GSBC_E_ARG, "desc.arrangement %u with %u streams is not a known arrangement", d->arrangement,
                    d->n_streams);
    if (d->n_pad != pad16(d->n_prims) || d->blocks_per_stream * streams_of(d->arrangement) != d->n_pad)
        return fail(ctx, GSBC_E_ARG, "desc sizes inconsistent (n_prims %llu, n_pad %llu, blocks per stream %llu)",
                    (unsigned long long)d->n_prims, (unsigned long long)d->n_pad, (unsigned long long)d->blocks_per_stream);
    return GSBC_OK;
}

gsbc_status check_stream(gsbc_ctx *ctx, const gsbc_stream_desc *d)
{
    gsbc_status s = check_desc(ctx, d);
    if (s) return s;
    uint64_t pos = 0;
    for (uint32_t k = 0; k < d->n_streams; k++) {
        if (!stream_format_ok(d->format[k], d->arrangement))
            return fail(ctx, GSBC_E_ARG, "desc.format[%u] = %u is not BC1, BC7 or (band streams) NONE", k, d->format[k]);
        if (d->offset[k] != pos) return fail(ctx, GSBC_E_ARG, "desc.offset[%u] does not follow the stream layout", k);
        pos = align16(pos + stream_bytes(d->format[k], d->blocks_per_stream));
    }
    if (d->payload_bytes != pos) return fail(ctx, GSBC_E_ARG, "desc.payload_bytes inconsistent");
    return GSBC_OK;
}

BandArgs band_args(const gsbc_stream_desc *d)
{
    BandArgs b;
    b.arrangement = d->arrangement;
    b.n_streams = d->n_streams;
    for (int k = 0; k < 16; k++) {
        const bool live = (uint32_t)k < d->n_streams;
        b.offset[k] = live ? d->offset[k] : 0;
        b.format[k] = live ? d->format[k] : 0;
        b.vmin[k] = d->vmin[k];
        b.delta[k] = (d->vmax[k] - d->vmin[k]) / 255.0f;
        const double d64 = ((double)d->vmax[k] - (double)d->vmin[k]) / 255.0;
        b.dhi[k] = (float)d64;
        b.dlo[k] = (float)(d64 - (double)b.dhi[k]);
    }
    return b;
}

char *small_ptr(gsbc_ctx *ctx, size_t off) { return static_cast<char *>(ctx->small) + off; }

// Block runs of one format, laid out in one global index space.
struct Runs {
    std::vector<BlockRun> v;
    uint64_t total = 0;
    void add(const uint8_t *src, uint8_t *dst, unsigned long long *sse, uint64_t nblk)
    {
        v.push_back({src, dst, sse, total, nblk});
        total += run_span(nblk);
    }
};

// Stream layout of the formats: stream k at offset[k], 16-byte aligned;
// entries past n_streams are zero.
uint64_t layout(const uint32_t fmt[16], uint32_t n_streams, uint64_t nblk, uint64_t off[16])
{
    uint64_t pos = 0;
    for (uint32_t k = n_streams; k < 16; k++) off[k] = 0;
    for (uint32_t k = 0; k < n_streams; k++) {
        off[k] = pos;
        pos = align16(pos + stream_bytes(fmt[k], nblk));
    }
    return pos;
}

// Arena bytes of one encode of nblk blocks per stream: [both candidate
// payloads (AUTO)] [BC7 runs] [BC1 runs] [BC7 key scratch]; AUTO is the
// largest (every band in both formats).
size_t encode_front_bytes(uint64_t nblk) { return 16 * align16(8 * nblk) + 16 * 16 * nblk; }
constexpr size_t kHistBytes = 16 * 256 * sizeof(uint64_t);   // band code histograms (the 0-bit option)

// Four-bit units of a rate target over S bands: rate*S/4, accepted within
// 1e-9 of an integer (a 9-band class scene has rates such as 44/9); -1 if not.
long rate_units(double rate, uint32_t S)
{
    const double u = rate * (double)S / 4.0;
    const double r = floor(u + 0.5);
    if (!(fabs(u - r) <= 1e-9) || r < 0.0 || r > 1e6) return -1;
    return (long)r;
}

// Default work split of the single-scene calls: one workgroup per 256-block
// round, BC1 on 128-lane workgroups, one BC7 search launch whose work items
// are (candidate group, round) pairs.
constexpr WorkSplit kPlainSplit = {1, 0, nullptr};
constexpr uint32_t kPlainBc1Lanes = 128;
constexpr uint32_t kPlainBc7Split = 3;
constexpr size_t kRunTableBytes = 16 * sizeof(BlockRun);   // one scene, one format
constexpr size_t kRunStageOff = 2048;                        // in ctx->pinned

// The second stream (default priority) and its fork/join events.
gsbc_status ensure_side(gsbc_ctx *ctx)
{
    if (ctx->side) return GSBC_OK;
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking), "side stream");
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming), "event");
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming), "event");
    return GSBC_OK;
}

void drop_plan(gsbc_ctx *ctx)
{
    // a replay of the plan may still be running on the stream
    if (ctx->graph_exec || ctx->plan_mem) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->plan_mem) (void)hipFree(ctx->plan_mem);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->plan_mem = nullptr;
    ctx->plan_sse = nullptr;
    ctx->plan_sig.clear();
}

}  // namespace

namespace gsbc {

void trace_begin(const char *kernel, hipStream_t st)
{
    gsbc_ctx *c = t_active;
    if (!c || !c->profiling || c->capturing) return;
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
    if (!c || !c->profiling || c->capturing || c->recs.empty()) return;
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
    p->order = 0;
    p->arrangement = GSBC_ARR_BANDS;
    p->quantiser = 0;
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
    {   // the range extremes start neutral: minima all ones, maxima zero
        uint32_t acc0[38];
        for (int i = 0; i < 38; i++) acc0[i] = (i < 16 || (i >= 32 && i < 35)) ? 0xFFFFFFFFu : 0u;
        if (hipMemset(ctx->small, 0, kSmallBytes) != hipSuccess ||
            hipMemcpy(static_cast<char *>(ctx->small) + kRangeOff + offsetof(RangeRec, acc), acc0, sizeof acc0,
                      hipMemcpyHostToDevice) != hipSuccess)
            return bail(GSBC_E_DEVICE);
    }
    if (hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault) != hipSuccess) return bail(GSBC_E_NOMEM);
    if (upload_bc1_tables(device, ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
    if (upload_bc7_tables(device, ctx->stream) != hipSuccess) return bail(GSBC_E_DEVICE);
    if (init_static_scratch(device) != hipSuccess) return bail(GSBC_E_DEVICE);
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
    drop_plan(ctx);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->arena) (void)hipFree(ctx->arena);
    for (void *p : ctx->retired) (void)hipFree(p);
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

gsbc_status gsbc_reserve(gsbc_ctx *ctx, uint64_t n_max, uint32_t n_dirs_max)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    if (n_max == 0 || n_max > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "n_max = %llu not in 1..2^31-1",
                                                         (unsigned long long)n_max);
    const uint64_t nblk = pad16(n_max) / 16;
    size_t need = reorder_scratch_bytes(n_max, 3);
    need = std::max(need, encode_front_bytes(nblk) + 2 * kRunTableBytes + bc7_scratch_bytes(16 * run_span(nblk)) +
                              kHistBytes);
    need = std::max(need, (size_t)n_dirs_max * 16 * sizeof(float));
    return ensure_arena(ctx, need);
}

gsbc_status gsbc_arena_info(const gsbc_ctx *ctx, uint64_t *bytes, uint64_t *growths)
{
    if (!ctx) return GSBC_E_ARG;
    if (bytes) *bytes = ctx->arena_bytes;
    if (growths) *growths = ctx->arena_growths;
    return GSBC_OK;
}

namespace {

// Wait for the stream, then desc from the range record of the last
// gsbc_reorder and its n and params (staged: that call's last kernel has
// already copied the record to the pinned block).
gsbc_status read_reorder_desc(gsbc_ctx *ctx, gsbc_stream_desc *desc, bool staged)
{
    const RangeRec *range = reinterpret_cast<const RangeRec *>(small_ptr(ctx, kRangeOff));
    if (!staged)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, range, sizeof(RangeRec), hipMemcpyDeviceToHost, ctx->stream),
                "range read-back");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "reorder");
    const RangeRec *r = static_cast<const RangeRec *>(ctx->pinned);
    const gsbc_params &p = ctx->last_p;
    const uint64_t n = ctx->last_n;
    memset(desc, 0, sizeof *desc);
    for (int k = 0; k < 16; k++) { desc->vmin[k] = r->vmin[k]; desc->vmax[k] = r->vmax[k]; }
    desc->n_prims = n;
    desc->n_pad = pad16(n);
    desc->arrangement = p.arrangement;
    desc->n_streams = streams_of(p.arrangement);
    desc->blocks_per_stream = desc->n_pad / desc->n_streams;
    return GSBC_OK;
}

}  // namespace

gsbc_status gsbc_reorder(gsbc_ctx *ctx, const float *pos, const float *sh, const float *opacity, uint64_t n,
                         const gsbc_params *params, uint32_t *perm, uint8_t *textures, gsbc_stream_desc *desc)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!pos || !sh || !perm || !textures) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (n == 0 || n > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "n = %llu not in 1..2^31-1", (unsigned long long)n);
    if ((reinterpret_cast<uintptr_t>(sh) & 15) || (reinterpret_cast<uintptr_t>(textures) & 15) ||
        (reinterpret_cast<uintptr_t>(pos) & 3) || (reinterpret_cast<uintptr_t>(perm) & 3) ||
        (reinterpret_cast<uintptr_t>(opacity) & 3))
        return fail(ctx, GSBC_E_ARG, "sh and textures must be 16-byte aligned, pos, opacity and perm 4-byte aligned");
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    if (p.quantiser == 1 && 3 * n > 0xFFFFFFFFull)
        return fail(ctx, GSBC_E_ARG, "quantiser 1 counts 3n coefficients per band in 32 bits: n = %llu too large",
                    (unsigned long long)n);
    if ((s = ensure_arena(ctx, reorder_scratch_bytes(n, p.grid_bits)))) return s;
    RangeRec *range = reinterpret_cast<RangeRec *>(small_ptr(ctx, kRangeOff));
    ctx->reordered = false;
    // with a desc, the last kernel also writes the range record to the pinned
    // staging block, so only a wait is left
    HIP_TRY(ctx, launch_reorder(pos, sh, opacity, n, p.grid_bits, p.quantiser, p.order == 1, p.arrangement, perm,
                                 textures, ctx->arena, range, desc ? static_cast<RangeRec *>(ctx->pinned) : nullptr,
                                 ctx->stream),
            "reorder launch");
    ctx->reordered = true;
    ctx->last_n = n;
    ctx->last_p = p;
    return desc ? read_reorder_desc(ctx, desc, true) : GSBC_OK;
}

gsbc_status gsbc_reorder_desc(gsbc_ctx *ctx, gsbc_stream_desc *desc)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!desc) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (!ctx->reordered) return fail(ctx, GSBC_E_ARG, "no gsbc_reorder on this context since the last range use");
    return read_reorder_desc(ctx, desc, false);
}

gsbc_status gsbc_reorder_degrees(gsbc_ctx *ctx, const float *pos, const float *sh, const float *opacity, uint64_t n,
                                 float tau, const gsbc_params *params, uint32_t *perm, uint8_t *textures,
                                 uint64_t textures_capacity, uint64_t counts[4], uint64_t tex_offset[4],
                                 gsbc_stream_desc descs[4])
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!pos || !sh || !perm || !textures || !counts || !tex_offset || !descs)
        return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (n == 0 || n > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "n = %llu not in 1..2^31-1", (unsigned long long)n);
    if ((reinterpret_cast<uintptr_t>(sh) & 15) || (reinterpret_cast<uintptr_t>(textures) & 15) ||
        (reinterpret_cast<uintptr_t>(pos) & 3) || (reinterpret_cast<uintptr_t>(perm) & 3) ||
        (reinterpret_cast<uintptr_t>(opacity) & 3))
        return fail(ctx, GSBC_E_ARG, "sh and textures must be 16-byte aligned, pos, opacity and perm 4-byte aligned");
    if (!(tau >= 0.0f) || !isfinite(tau)) return fail(ctx, GSBC_E_ARG, "tau must be finite and >= 0");
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    if (p.order != 0 || (p.arrangement != GSBC_ARR_BANDS && p.arrangement != GSBC_ARR_QUAD))
        return fail(ctx, GSBC_E_ARG,
                    "degree classes are sorted (order 0) in band streams (GSBC_ARR_BANDS) or with the degree-1 "
                    "class in Fig. SetupC (GSBC_ARR_QUAD)");
    const bool setup_c = p.arrangement == GSBC_ARR_QUAD;
    if (p.quantiser == 1 && 3 * n > 0xFFFFFFFFull)
        return fail(ctx, GSBC_E_ARG, "quantiser 1 counts 3n coefficients per band in 32 bits: n = %llu too large",
                    (unsigned long long)n);
    const uint64_t need = degree_textures_bytes(n);
    if (textures_capacity < need)
        return fail(ctx, GSBC_E_BUFFER, "textures_capacity %llu < %llu bytes", (unsigned long long)textures_capacity,
                    (unsigned long long)need);
    if ((s = ensure_arena(ctx, reorder_scratch_bytes(n, p.grid_bits)))) return s;
    RangeRec *range = reinterpret_cast<RangeRec *>(small_ptr(ctx, kRangeOff));
    uint32_t *cls = reinterpret_cast<uint32_t *>(small_ptr(ctx, kClassOff));
    ctx->reordered = false;   // the range record is this call's now
    HIP_TRY(ctx, launch_degree_sort(pos, sh, opacity, n, p.grid_bits, p.quantiser, tau, perm, ctx->arena, range, cls,
                                    ctx->stream), "degree sort launch");
    char *stage = static_cast<char *>(ctx->pinned);
    HIP_TRY(ctx, hipMemcpyAsync(stage, range, sizeof(RangeRec), hipMemcpyDeviceToHost, ctx->stream), "range read-back");
    HIP_TRY(ctx, hipMemcpyAsync(stage + 512, cls, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream),
            "class counts");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "degree sort");
    RangeRec r;
    memcpy(&r, stage, sizeof r);
    uint32_t c32[4];
    memcpy(c32, stage + 512, sizeof c32);
    DegreeLayout lay;
    lay.slot_start[0] = lay.pad_start[0] = 0;
    uint64_t word = 0;
    for (int L = 0; L < 4; L++) {
        counts[L] = c32[L];
        lay.slot_start[L + 1] = lay.slot_start[L] + c32[L];
        lay.pad_start[L + 1] = lay.pad_start[L] + pad16(c32[L]);
        lay.tex_word[L] = word;
        tex_offset[L] = word * 4;
        word += (uint64_t)(L + 1) * (L + 1) * pad16(c32[L]);    // (L+1)^2 streams of pad16/16 blocks x 16 words
    }
    if (lay.slot_start[4] != n) return fail(ctx, GSBC_E_DEVICE, "class counts do not add up to n");
    lay.quad1 = setup_c ? 1u : 0u;
    HIP_TRY(ctx, launch_pack_degrees(sh, opacity, perm, lay, range, textures, ctx->stream), "degree pack launch");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "degree pack");
    for (int L = 0; L < 4; L++) {
        gsbc_stream_desc &d = descs[L];
        memset(&d, 0, sizeof d);
        for (int k = 0; k < 16; k++) { d.vmin[k] = r.vmin[k]; d.vmax[k] = r.vmax[k]; }
        d.n_prims = counts[L];
        d.n_pad = pad16(counts[L]);
        if (setup_c && L == 1) {   // one stream of n_pad/4 blocks, four primitives each
            d.arrangement = GSBC_ARR_QUAD;
            d.n_streams = 1;
            d.blocks_per_stream = d.n_pad / 4;
        } else {
            d.arrangement = GSBC_ARR_BANDS;
            d.n_streams = (uint32_t)((L + 1) * (L + 1));
            d.blocks_per_stream = d.n_pad / 16;
        }
    }
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
    if (format != GSBC_FMT_AUTO && format != GSBC_FMT_AUTO_ZERO && format != GSBC_FMT_BC1 && format != GSBC_FMT_BC7 &&
        format != GSBC_FMT_BANDS)
        return fail(ctx, GSBC_E_ARG, "format %d is not AUTO(0), BC1(1), BANDS(2), AUTO_ZERO(4) or BC7(7)", format);
    const uint32_t S = desc->n_streams;
    const bool autoc = format == GSBC_FMT_AUTO || format == GSBC_FMT_AUTO_ZERO;
    if (format == GSBC_FMT_BANDS)
        for (uint32_t k = 0; k < S; k++)
            if (!stream_format_ok(desc->format[k], desc->arrangement))
                return fail(ctx, GSBC_E_ARG, "desc.format[%u] = %u is not BC1, BC7 or (band streams) NONE", k,
                            desc->format[k]);
    if (autoc && desc->arrangement != GSBC_ARR_BANDS)
        return fail(ctx, GSBC_E_UNSUPPORTED, "the rate controller chooses per band: GSBC_ARR_BANDS scenes only");
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    const uint64_t nblk = desc->blocks_per_stream;
    unsigned long long *sse1 = reinterpret_cast<unsigned long long *>(small_ptr(ctx, kSse1Off));
    unsigned long long *sse7 = reinterpret_cast<unsigned long long *>(small_ptr(ctx, kSse7Off));
    const uint64_t tex_band = nblk * 64;

    uint64_t host_off[16];
    uint32_t host_fmt[16];
    uint64_t payload = 0;
    uint32_t k_auto = 0;   // AUTO: bands upgraded to BC7; AUTO_ZERO: units over bands 1..S-1
    bool have1 = false, have7 = false;
    Runs r1, r7;
    uint8_t *buf1 = nullptr, *buf7 = nullptr;
    uint64_t off1[16], off7[16];
    size_t front = 0;
    if (!autoc) {
        for (uint32_t k = 0; k < 16; k++)
            host_fmt[k] = k >= S ? 0u : format == GSBC_FMT_BANDS ? desc->format[k] : (uint32_t)format;
        payload = layout(host_fmt, S, nblk, host_off);
        if (blocks_capacity < payload)
            return fail(ctx, GSBC_E_BUFFER, "blocks_capacity %llu < payload %llu bytes", (unsigned long long)blocks_capacity,
                        (unsigned long long)payload);
        for (uint32_t k = 0; k < S; k++) {
            if (host_fmt[k] == GSBC_FMT_BC7) r7.add(textures + k * tex_band, blocks + host_off[k], sse7 + k, nblk);
            else if (host_fmt[k] == GSBC_FMT_BC1) r1.add(textures + k * tex_band, blocks + host_off[k], sse1 + k, nblk);
        }
    } else {
        const long units = rate_units(rate, S);
        if (format == GSBC_FMT_AUTO) {
            const long k = units - (long)S - 1;
            if (units < 0 || k < 0 || k > (long)S - 1)
                return fail(ctx, GSBC_E_INFEASIBLE,
                            "rate %.17g bits/texel over %u bands needs rate*S/4 - S - 1 BC7 bands, not an integer in 0..%u",
                            rate, S, S - 1);
            k_auto = (uint32_t)k;
            payload = (uint64_t)(k_auto + 1) * 16 * nblk + (uint64_t)(S - 1 - k_auto) * align16(8 * nblk);
        } else {
            const long U = units - 2;
            if (units < 0 || U < 0 || U > 2 * ((long)S - 1))
                return fail(ctx, GSBC_E_INFEASIBLE,
                            "rate %.17g bits/texel over %u bands needs rate*S/4 - 2 units, not an integer in 0..%u", rate, S,
                            2 * (S - 1));
            k_auto = (uint32_t)U;
            // the largest payload of any choice with U units (BC1 streams pad to 16 bytes)
            for (long n7 = U > (long)S - 1 ? U - ((long)S - 1) : 0; 2 * n7 <= U; n7++)
                payload = std::max<uint64_t>(payload, (uint64_t)(1 + n7) * 16 * nblk + (uint64_t)(U - 2 * n7) * align16(8 * nblk));
        }
        if (blocks_capacity < payload)
            return fail(ctx, GSBC_E_BUFFER, "blocks_capacity %llu < payload %llu bytes", (unsigned long long)blocks_capacity,
                        (unsigned long long)payload);
        front = encode_front_bytes(nblk);   // both candidate payloads
    }
    // arena: [candidate payloads (AUTO)] [BC7 runs] [BC1 runs] [BC7 key scratch] [band histograms (AUTO_ZERO)]
    const uint64_t total7 = autoc ? (uint64_t)S * run_span(nblk) : r7.total;
    const size_t hist_off = front + 2 * kRunTableBytes + bc7_scratch_bytes(total7);
    if ((s = ensure_arena(ctx, hist_off + (format == GSBC_FMT_AUTO_ZERO ? kHistBytes : 0)))) return s;
    uint8_t *arena = static_cast<uint8_t *>(ctx->arena);
    if (autoc) {
        buf1 = arena;
        buf7 = buf1 + 16 * align16(8 * nblk);
        for (int q = 0; q < 16; q++) {
            off1[q] = q * align16(8 * nblk);
            off7[q] = q * 16 * nblk;
        }
        for (uint32_t q = 0; q < S; q++) {
            r7.add(textures + q * tex_band, buf7 + off7[q], sse7 + q, nblk);
            r1.add(textures + q * tex_band, buf1 + off1[q], sse1 + q, nblk);   // band 0 too: its BC1 SSE is reported
        }
    }
    BlockRun *druns7 = reinterpret_cast<BlockRun *>(arena + front);
    BlockRun *druns1 = druns7 + 16;
    have1 = !r1.v.empty();
    have7 = !r7.v.empty();
    char *stage = static_cast<char *>(ctx->pinned) + kRunStageOff;
    memcpy(stage, r7.v.data(), r7.v.size() * sizeof(BlockRun));
    memcpy(stage + kRunTableBytes, r1.v.data(), r1.v.size() * sizeof(BlockRun));
    HIP_TRY(ctx, hipMemcpyAsync(druns7, stage, 2 * kRunTableBytes, hipMemcpyHostToDevice, ctx->stream), "run tables");
    HIP_TRY(ctx, launch_fill_u64(sse1, 32, 0, ctx->stream), "clear");
    EncodeArgs a;
    memset(&a, 0, sizeof a);
    a.refine_steps = p.refine_steps;
    a.mode_mask = p.bc7_mode_mask;
    a.keys = reinterpret_cast<uint32_t *>(arena + front + 2 * kRunTableBytes);
    const WorkSplit w3[3] = {kPlainSplit, kPlainSplit, kPlainSplit};
    // With both formats: the BC7 search runs alone on the context's stream
    // (its device time is its own), then the BC1 encoder runs on a side
    // stream beside the short, latency-bound BC7 bucketing and emit kernels,
    // joined before anything reads either format's results.  While kernel
    // timing is on, everything stays on the context's stream, one kernel
    // after another, so each timed kernel has the GPU to itself.
    hipStream_t s1 = ctx->stream;
    const bool both = have1 && have7 && !ctx->profiling;
    if (both) {
        if ((s = ensure_side(ctx))) return s;
        s1 = ctx->side;
    }
    if (have7) {
        a.run = druns7;
        a.nrun = (uint32_t)r7.v.size();
        a.total = r7.total;
        HIP_TRY(ctx, launch_bc7_encode(a, w3, kPlainBc7Split, ctx->stream, both ? ctx->fork : nullptr), "bc7 launch");
    }
    if (have1) {
        EncodeArgs a1 = a;
        a1.run = druns1;
        a1.nrun = (uint32_t)r1.v.size();
        a1.total = r1.total;
        if (both) HIP_TRY(ctx, hipStreamWaitEvent(s1, ctx->fork, 0), "fork");
        HIP_TRY(ctx, launch_bc1_encode(a1, kPlainSplit, kPlainBc1Lanes, s1), "bc1 launch");
    }
    if (s1 != ctx->stream) {
        HIP_TRY(ctx, hipEventRecord(ctx->join, s1), "join");
        HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, ctx->join, 0), "join");
    }
    if (autoc) {
        uint64_t *doff1 = reinterpret_cast<uint64_t *>(small_ptr(ctx, kOff1Off));
        uint64_t *doff7 = reinterpret_cast<uint64_t *>(small_ptr(ctx, kOff7Off));
        uint64_t *ostage = reinterpret_cast<uint64_t *>(static_cast<char *>(ctx->pinned) + kRunStageOff + 2 * kRunTableBytes);
        memcpy(ostage, off1, sizeof off1);
        memcpy(ostage + 16, off7, sizeof off7);
        HIP_TRY(ctx, hipMemcpyAsync(doff1, ostage, 2 * sizeof off1, hipMemcpyHostToDevice, ctx->stream), "offsets");
        RateSel *sel = reinterpret_cast<RateSel *>(small_ptr(ctx, kSelOff));
        if (format == GSBC_FMT_AUTO_ZERO) {
            unsigned long long *hist = reinterpret_cast<unsigned long long *>(arena + hist_off);
            HIP_TRY(ctx, launch_fill_u64(hist, 16 * 256, 0, ctx->stream), "clear");
            HIP_TRY(ctx, launch_band_hist(textures, S, nblk, hist, ctx->stream), "band histograms");
            HIP_TRY(ctx, launch_rate_select_zero(sse1, sse7, hist, band_args(desc), S, k_auto, nblk, sel, ctx->stream),
                    "rate select");
        } else {
            HIP_TRY(ctx, launch_rate_select(sse1, sse7, band_args(desc), S, k_auto, nblk, sel, ctx->stream), "rate select");
        }
        HIP_TRY(ctx, launch_copy_streams(buf1, doff1, buf7, doff7, sel, S, nblk, blocks, ctx->stream), "stream copy");
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, sel, sizeof(RateSel), hipMemcpyDeviceToHost, ctx->stream), "selection read-back");
    }
    char *sstage = static_cast<char *>(ctx->pinned) + 1024;
    HIP_TRY(ctx, hipMemcpyAsync(sstage, sse1, 32 * sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream), "sse read-back");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "encode");
    if (autoc) {
        const RateSel *r = static_cast<const RateSel *>(ctx->pinned);
        for (int q = 0; q < 16; q++) { host_fmt[q] = r->format[q]; host_off[q] = r->offset[q]; }
        if (format == GSBC_FMT_AUTO ? r->payload_bytes != payload : r->payload_bytes > payload)
            return fail(ctx, GSBC_E_DEVICE, "selected payload size disagrees with the budget");
        payload = r->payload_bytes;
    }
    if (band_sse) {
        const uint64_t *h = reinterpret_cast<const uint64_t *>(sstage);
        for (uint32_t q = 0; q < 16; q++) {
            const bool c1 = q < S && (autoc || (have1 && host_fmt[q] == GSBC_FMT_BC1));
            const bool c7 = q < S && (autoc || (have7 && host_fmt[q] == GSBC_FMT_BC7));
            band_sse[q] = c1 ? (int64_t)h[q] : -1;
            band_sse[16 + q] = c7 ? (int64_t)h[16 + q] : -1;
        }
    }
    for (int q = 0; q < 16; q++) { desc->format[q] = (uint8_t)host_fmt[q]; desc->offset[q] = host_off[q]; }
    desc->payload_bytes = payload;
    return GSBC_OK;
}

void gsbc_default_batch_tuning(gsbc_batch_tuning *t)
{
    if (!t) return;
    t->item_rounds = 1;
    t->wgs_per_cu = 0;
    t->bc1_lanes = kPlainBc1Lanes;
    t->bc7_split = kPlainBc7Split;
    t->concurrent = 0;
}

gsbc_status gsbc_encode_batch(gsbc_ctx *ctx, uint32_t n_scenes, const uint8_t *const *textures,
                              gsbc_stream_desc *descs, uint8_t *const *blocks, const uint64_t *blocks_capacity,
                              const gsbc_params *params, const gsbc_batch_tuning *tuning, int64_t *band_sse)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!textures || !descs || !blocks || !blocks_capacity) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (n_scenes == 0 || n_scenes > 4096) return fail(ctx, GSBC_E_ARG, "n_scenes %u not in 1..4096", n_scenes);
    gsbc_params p = resolve(params);
    if ((s = check_params(ctx, p))) return s;
    gsbc_batch_tuning t;
    gsbc_default_batch_tuning(&t);
    if (tuning) t = *tuning;
    if (t.item_rounds < 1 || t.item_rounds > 64) return fail(ctx, GSBC_E_ARG, "tuning.item_rounds %u not in 1..64", t.item_rounds);
    if (t.wgs_per_cu > 16) return fail(ctx, GSBC_E_ARG, "tuning.wgs_per_cu %u > 16", t.wgs_per_cu);
    if (t.bc1_lanes != 64 && t.bc1_lanes != 128 && t.bc1_lanes != 256)
        return fail(ctx, GSBC_E_ARG, "tuning.bc1_lanes %u is not 64, 128 or 256", t.bc1_lanes);
    if (t.bc7_split > 3) return fail(ctx, GSBC_E_ARG, "tuning.bc7_split %u > 3", t.bc7_split);
    if (t.concurrent > 1) return fail(ctx, GSBC_E_ARG, "tuning.concurrent %u > 1", t.concurrent);
    // validate every scene and lay out its streams (host only, nothing enqueued yet)
    std::vector<uint64_t> offs(16 * (size_t)n_scenes), pay(n_scenes);
    std::vector<uint32_t> fmts(16 * (size_t)n_scenes);
    for (uint32_t i = 0; i < n_scenes; i++) {
        if (!textures[i] || !blocks[i]) return fail(ctx, GSBC_E_ARG, "scene %u: NULL pointer", i);
        if ((reinterpret_cast<uintptr_t>(textures[i]) & 15) || (reinterpret_cast<uintptr_t>(blocks[i]) & 15))
            return fail(ctx, GSBC_E_ARG, "scene %u: textures and blocks must be 16-byte aligned", i);
        if ((s = check_desc(ctx, &descs[i]))) return s;
        for (uint32_t k = 0; k < 16; k++) {
            fmts[16 * i + k] = k < descs[i].n_streams ? descs[i].format[k] : 0u;
            if (k < descs[i].n_streams && !stream_format_ok(fmts[16 * i + k], descs[i].arrangement))
                return fail(ctx, GSBC_E_ARG, "scene %u: desc.format[%u] = %u is not BC1, BC7 or (band streams) NONE", i, k,
                            descs[i].format[k]);
        }
        pay[i] = layout(&fmts[16 * i], descs[i].n_streams, descs[i].blocks_per_stream, &offs[16 * i]);
        if (blocks_capacity[i] < pay[i])
            return fail(ctx, GSBC_E_BUFFER, "scene %u: blocks_capacity %llu < payload %llu bytes", i,
                        (unsigned long long)blocks_capacity[i], (unsigned long long)pay[i]);
    }
    // the plan signature: everything the captured launches depend on
    std::vector<uint64_t> sig;
    sig.reserve(8 + 20 * (size_t)n_scenes);
    sig.push_back(n_scenes);
    sig.push_back(p.refine_steps);
    sig.push_back(p.bc7_mode_mask);
    sig.push_back(((uint64_t)t.item_rounds << 32) | t.wgs_per_cu);
    sig.push_back(((uint64_t)t.bc1_lanes << 32) | (t.bc7_split << 1) | t.concurrent);
    for (uint32_t i = 0; i < n_scenes; i++) {
        sig.push_back(reinterpret_cast<uintptr_t>(textures[i]));
        sig.push_back(reinterpret_cast<uintptr_t>(blocks[i]));
        sig.push_back(descs[i].blocks_per_stream);
        uint64_t f = (uint64_t)descs[i].n_streams << 32;
        for (int k = 0; k < 16; k++)
            f |= (uint64_t)(fmts[16 * i + k] == GSBC_FMT_BC7 ? 2 : fmts[16 * i + k] == GSBC_FMT_NONE ? 3 : 1) << (2 * k);
        sig.push_back(f);
    }
    if (sig != ctx->plan_sig) {
        drop_plan(ctx);
        Runs r1, r7;
        for (uint32_t i = 0; i < n_scenes; i++) {
            const uint64_t nblk = descs[i].blocks_per_stream;
            for (uint32_t k = 0; k < descs[i].n_streams; k++) {
                const uint8_t *src = textures[i] + (uint64_t)k * nblk * 64;
                uint8_t *dst = blocks[i] + offs[16 * i + k];
                if (fmts[16 * i + k] == GSBC_FMT_BC7) r7.add(src, dst, nullptr, nblk);
                else if (fmts[16 * i + k] == GSBC_FMT_BC1) r1.add(src, dst, nullptr, nblk);
            }
        }
        // plan memory: [runs7][runs1][sse n_scenes x 16][queues 4 x u64][BC7 keys]
        const size_t b7 = align16(r7.v.size() * sizeof(BlockRun)), b1 = align16(r1.v.size() * sizeof(BlockRun));
        const size_t bs = 16 * (size_t)n_scenes * 8, bq = 64;
        const size_t bytes = b7 + b1 + bs + bq + bc7_scratch_bytes(r7.total);
        if (injected_alloc_failure()) return fail(ctx, GSBC_E_NOMEM, "plan allocation of %zu bytes failed (injected)", bytes);
        hipError_t e = hipMalloc(&ctx->plan_mem, bytes);
        if (e != hipSuccess) {
            ctx->plan_mem = nullptr;
            (void)hipGetLastError();
            return fail(ctx, GSBC_E_NOMEM, "plan allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        }
        uint8_t *pm = static_cast<uint8_t *>(ctx->plan_mem);
        BlockRun *d7 = reinterpret_cast<BlockRun *>(pm), *d1 = reinterpret_cast<BlockRun *>(pm + b7);
        ctx->plan_sse = reinterpret_cast<unsigned long long *>(pm + b7 + b1);
        uint32_t *queues = reinterpret_cast<uint32_t *>(pm + b7 + b1 + bs);
        uint32_t *keys = reinterpret_cast<uint32_t *>(pm + b7 + b1 + bs + bq);
        {   // each run adds into its (scene, band) SSE slot
            size_t q7 = 0, q1 = 0;
            for (uint32_t i = 0; i < n_scenes; i++)
                for (uint32_t k = 0; k < descs[i].n_streams; k++) {
                    if (fmts[16 * i + k] == GSBC_FMT_NONE) continue;
                    BlockRun &r = fmts[16 * i + k] == GSBC_FMT_BC7 ? r7.v[q7++] : r1.v[q1++];
                    r.sse = ctx->plan_sse + 16 * (size_t)i + k;
                }
        }
        if (!r7.v.empty()) HIP_TRY(ctx, hipMemcpy(d7, r7.v.data(), r7.v.size() * sizeof(BlockRun), hipMemcpyHostToDevice), "run table");
        if (!r1.v.empty()) HIP_TRY(ctx, hipMemcpy(d1, r1.v.data(), r1.v.size() * sizeof(BlockRun), hipMemcpyHostToDevice), "run table");
        int cus = 0;
        HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device), "device attribute");
        if (t.concurrent && (s = ensure_side(ctx))) return s;
        EncodeArgs a;
        memset(&a, 0, sizeof a);
        a.refine_steps = p.refine_steps;
        a.mode_mask = p.bc7_mode_mask;
        a.keys = keys;
        WorkSplit w3[3], w1;
        for (int q = 0; q < 3; q++)
            w3[q] = {t.item_rounds, (uint32_t)cus * t.wgs_per_cu, t.wgs_per_cu ? queues + 2 * q : nullptr};
        w1 = {t.item_rounds, (uint32_t)cus * t.wgs_per_cu, t.wgs_per_cu ? queues + 6 : nullptr};
        // capture the whole sequence once
        ctx->capturing = true;
        e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { ctx->capturing = false; drop_plan(ctx); return hip_fail(ctx, e, "graph capture"); }
        hipError_t le = launch_fill_u64(ctx->plan_sse, 16 * (uint64_t)n_scenes, 0, ctx->stream);
        hipStream_t s1 = ctx->stream;
        if (le == hipSuccess && t.concurrent && !r1.v.empty() && !r7.v.empty()) {
            le = hipEventRecord(ctx->fork, ctx->stream);
            if (le == hipSuccess) le = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
            s1 = ctx->side;
        }
        if (le == hipSuccess && !r7.v.empty()) {
            a.run = d7;
            a.nrun = (uint32_t)r7.v.size();
            a.total = r7.total;
            le = launch_bc7_encode(a, w3, t.bc7_split, ctx->stream);
        }
        if (le == hipSuccess && !r1.v.empty()) {
            a.run = d1;
            a.nrun = (uint32_t)r1.v.size();
            a.total = r1.total;
            le = launch_bc1_encode(a, w1, t.bc1_lanes, s1);
        }
        if (le == hipSuccess && s1 != ctx->stream) {
            le = hipEventRecord(ctx->join, s1);
            if (le == hipSuccess) le = hipStreamWaitEvent(ctx->stream, ctx->join, 0);
        }
        e = hipStreamEndCapture(ctx->stream, &ctx->graph);
        ctx->capturing = false;
        if (le != hipSuccess || e != hipSuccess) {
            drop_plan(ctx);
            return hip_fail(ctx, le != hipSuccess ? le : e, "batch capture");
        }
        e = hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_plan(ctx); return hip_fail(ctx, e, "graph instantiate"); }
        ctx->plan_sig = sig;
    }
    trace_begin("encode_batch_graph", ctx->stream);
    HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream), "graph launch");
    trace_end(ctx->stream);
    for (uint32_t i = 0; i < n_scenes; i++) {
        for (int k = 0; k < 16; k++) descs[i].offset[k] = offs[16 * i + k];
        descs[i].payload_bytes = pay[i];
    }
    if (band_sse) {
        std::vector<uint64_t> h(16 * (size_t)n_scenes);
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "encode_batch");
        HIP_TRY(ctx, hipMemcpy(h.data(), ctx->plan_sse, h.size() * 8, hipMemcpyDeviceToHost), "sse read-back");
        for (size_t q = 0; q < h.size(); q++) band_sse[q] = (int64_t)h[q];
    }
    return GSBC_OK;
}

// ---- container files
namespace {
constexpr uint32_t kContainerVersion = 2;   // 1: before arrangements (always GSBC_ARR_BANDS)
constexpr uint32_t kRecordBytes = 24;

struct FileCloser {
    FILE *f;
    ~FileCloser() { if (f) fclose(f); }
};

void put32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
void put64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
uint32_t get32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
uint64_t get64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
}  // namespace

gsbc_status gsbc_save(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc, const char *path)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!blocks || !desc || !path) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if ((s = check_stream(ctx, desc))) return s;
    std::vector<uint8_t> buf(64 + 16 * kRecordBytes + desc->payload_bytes, 0);
    memcpy(buf.data(), "GSBC", 4);
    put32(&buf[4], kContainerVersion);
    put64(&buf[8], desc->n_prims);
    put64(&buf[16], desc->n_pad);
    put64(&buf[24], desc->blocks_per_stream);
    put64(&buf[32], desc->payload_bytes);
    put32(&buf[40], kRecordBytes);
    put32(&buf[44], desc->arrangement);
    put32(&buf[48], desc->n_streams);
    for (uint32_t k = 0; k < 16; k++) {
        uint8_t *r = &buf[64 + k * kRecordBytes];
        put32(r, k < desc->n_streams ? desc->format[k] : 0u);
        put64(r + 8, k < desc->n_streams ? desc->offset[k] : 0u);
        memcpy(r + 16, &desc->vmin[k], 4);
        memcpy(r + 20, &desc->vmax[k], 4);
    }
    HIP_TRY(ctx, hipMemcpyAsync(&buf[64 + 16 * kRecordBytes], blocks, desc->payload_bytes, hipMemcpyDeviceToHost,
                                ctx->stream), "payload read-back");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "save");
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) return fail(ctx, GSBC_E_IO, "cannot open %s for writing", path);
    if (fwrite(buf.data(), 1, buf.size(), fc.f) != buf.size() || fflush(fc.f) != 0)
        return fail(ctx, GSBC_E_IO, "short write to %s", path);
    return GSBC_OK;
}

gsbc_status gsbc_load(gsbc_ctx *ctx, const char *path, gsbc_stream_desc *desc, uint8_t *blocks, uint64_t blocks_capacity)
{
    if (blocks) {
        gsbc_status s = begin(ctx);
        if (s) return s;
    } else if (ctx) {
        ctx->err[0] = 0;
    }
    if (!path || !desc) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return fail(ctx, GSBC_E_IO, "cannot open %s", path);
    uint8_t head[64 + 16 * kRecordBytes];
    if (fread(head, 1, sizeof head, fc.f) != sizeof head) return fail(ctx, GSBC_E_IO, "%s: short header", path);
    if (memcmp(head, "GSBC", 4) != 0) return fail(ctx, GSBC_E_IO, "%s: not a container (bad magic)", path);
    const uint32_t version = get32(&head[4]);
    if (version != 1 && version != kContainerVersion) return fail(ctx, GSBC_E_IO, "%s: version %u not supported", path, version);
    if (get32(&head[40]) != kRecordBytes) return fail(ctx, GSBC_E_IO, "%s: record size %u", path, get32(&head[40]));
    gsbc_stream_desc d;
    memset(&d, 0, sizeof d);
    d.n_prims = get64(&head[8]);
    d.n_pad = get64(&head[16]);
    d.blocks_per_stream = get64(&head[24]);
    d.payload_bytes = get64(&head[32]);
    d.arrangement = version == 1 ? (uint32_t)GSBC_ARR_BANDS : get32(&head[44]);
    d.n_streams = version == 1 ? 16u : get32(&head[48]);
    for (int k = 0; k < 16; k++) {
        const uint8_t *r = &head[64 + k * kRecordBytes];
        const uint32_t f = get32(r);
        d.format[k] = (uint8_t)(f <= 255 ? f : 0);
        d.offset[k] = get64(r + 8);
        memcpy(&d.vmin[k], r + 16, 4);
        memcpy(&d.vmax[k], r + 20, 4);
    }
    gsbc_ctx scratch_ctx;
    if (check_stream(ctx ? ctx : &scratch_ctx, &d) != GSBC_OK)
        return fail(ctx, GSBC_E_IO, "%s: inconsistent header (%s)", path, ctx ? ctx->err : scratch_ctx.err);
    // the file holds exactly the header, the records and the payload
    if (fseek(fc.f, 0, SEEK_END) != 0) return fail(ctx, GSBC_E_IO, "%s: cannot seek", path);
    const long size = ftell(fc.f);
    if (size < 0 || (uint64_t)size != sizeof head + d.payload_bytes)
        return fail(ctx, GSBC_E_IO, "%s: %ld bytes, expected %llu", path, size,
                    (unsigned long long)(sizeof head + d.payload_bytes));
    if (fseek(fc.f, (long)sizeof head, SEEK_SET) != 0) return fail(ctx, GSBC_E_IO, "%s: cannot seek", path);
    if (blocks) {
        if (blocks_capacity < d.payload_bytes)
            return fail(ctx, GSBC_E_BUFFER, "blocks_capacity %llu < payload %llu bytes", (unsigned long long)blocks_capacity,
                        (unsigned long long)d.payload_bytes);
        std::vector<uint8_t> buf(d.payload_bytes);
        if (fread(buf.data(), 1, buf.size(), fc.f) != buf.size()) return fail(ctx, GSBC_E_IO, "%s: short payload", path);
        ActiveGuard guard(ctx);
        HIP_TRY(ctx, hipMemcpyAsync(blocks, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream), "payload upload");
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "load");
    }
    *desc = d;
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
    HIP_TRY(ctx, launch_decode(blocks, band_args(desc), desc->blocks_per_stream, textures_out, ctx->stream),
            "decode launch");
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

gsbc_status gsbc_decode_eval_noalloc(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                                     const float *dirs, uint32_t n_dirs, const uint32_t *prim_idx, uint64_t m,
                                     float *out)
{
    // the same checks and kernels as gsbc_decode_eval, with the basis rows in
    // the library's static device array instead of the context's arena: no
    // allocation of any kind (and no kernel timing, whose events would be)
    gsbc_status s = begin(ctx);
    if (s) return s;
    if (!blocks || !dirs || !out) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (reinterpret_cast<uintptr_t>(blocks) & 15) return fail(ctx, GSBC_E_ARG, "blocks must be 16-byte aligned");
    if ((reinterpret_cast<uintptr_t>(dirs) & 3) || (reinterpret_cast<uintptr_t>(out) & 3) ||
        (reinterpret_cast<uintptr_t>(prim_idx) & 3))
        return fail(ctx, GSBC_E_ARG, "dirs, prim_idx and out must be 4-byte aligned");
    if ((s = check_stream(ctx, desc))) return s;
    if (n_dirs == 0) return fail(ctx, GSBC_E_ARG, "n_dirs must be >= 1");
    if (n_dirs > kStaticScratchDirs)
        return fail(ctx, GSBC_E_ARG, "n_dirs %u exceeds the %u directions of the allocation-free scratch", n_dirs,
                    kStaticScratchDirs);
    if (m == 0) return fail(ctx, GSBC_E_ARG, "m must be >= 1");
    if (!prim_idx && m != desc->n_prims) return fail(ctx, GSBC_E_ARG, "prim_idx NULL requires m == n_prims");
    if (m > 0xFFFFFFFFull * 256) return fail(ctx, GSBC_E_ARG, "m too large");
    float *basis = static_scratch(ctx->device);
    if (!basis) return fail(ctx, GSBC_E_DEVICE, "static scratch of device %d not set up", ctx->device);
    HIP_TRY(ctx, launch_decode_eval(blocks, band_args(desc), desc->n_prims, dirs, n_dirs, prim_idx, m, out, basis,
                                    ctx->stream), "decode_eval launch");
    return GSBC_OK;
}

gsbc_status gsbc_decode_eval_view(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc, const float *pos,
                                  const uint32_t *perm, const float *view, const uint32_t *prim_idx, uint64_t m,
                                  float *out)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!blocks || !pos || !perm || !view || !out) return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (reinterpret_cast<uintptr_t>(blocks) & 15) return fail(ctx, GSBC_E_ARG, "blocks must be 16-byte aligned");
    if ((reinterpret_cast<uintptr_t>(pos) & 3) || (reinterpret_cast<uintptr_t>(perm) & 3) ||
        (reinterpret_cast<uintptr_t>(out) & 3) || (reinterpret_cast<uintptr_t>(prim_idx) & 3))
        return fail(ctx, GSBC_E_ARG, "pos, perm, prim_idx and out must be 4-byte aligned");
    if ((s = check_stream(ctx, desc))) return s;
    if (m == 0) return fail(ctx, GSBC_E_ARG, "m must be >= 1");
    if (!prim_idx && m != desc->n_prims) return fail(ctx, GSBC_E_ARG, "prim_idx NULL requires m == n_prims");
    if (m > 0xFFFFFFFFull * 256) return fail(ctx, GSBC_E_ARG, "m too large");
    const float f[3] = {view[0], view[1], view[2]};
    if (!(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]))) return fail(ctx, GSBC_E_ARG, "view position not finite");
    HIP_TRY(ctx, launch_decode_eval_view(blocks, band_args(desc), desc->n_prims, pos, perm, f, prim_idx, m, out,
                                         ctx->stream), "decode_eval_view launch");
    return GSBC_OK;
}

gsbc_status gsbc_blend_tiles(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc, const float *pos,
                             const uint32_t *perm, const float *view, const float *opacity, const float *footprint,
                             const uint32_t *tile_start, const uint32_t *list, uint64_t list_len, uint32_t tiles_x,
                             uint32_t tiles_y, float *image, float *transmittance)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!blocks || !pos || !perm || !view || !opacity || !footprint || !tile_start || !image || (!list && list_len))
        return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    if (reinterpret_cast<uintptr_t>(blocks) & 15) return fail(ctx, GSBC_E_ARG, "blocks must be 16-byte aligned");
    for (const void *q : {(const void *)pos, (const void *)perm, (const void *)opacity, (const void *)footprint,
                          (const void *)tile_start, (const void *)list, (const void *)image, (const void *)transmittance})
        if (reinterpret_cast<uintptr_t>(q) & 3) return fail(ctx, GSBC_E_ARG, "device arrays must be 4-byte aligned");
    if ((s = check_stream(ctx, desc))) return s;
    const uint64_t tiles = (uint64_t)tiles_x * tiles_y;
    if (tiles == 0 || tiles > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "%u x %u tiles", tiles_x, tiles_y);
    const float f[3] = {view[0], view[1], view[2]};
    if (!(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]))) return fail(ctx, GSBC_E_ARG, "view position not finite");
    if ((s = ensure_arena(ctx, tiles * sizeof(uint32_t)))) return s;   // the tile schedule
    HIP_TRY(ctx, launch_blend_tiles(blocks, band_args(desc), desc->n_prims, pos, perm, f, opacity, footprint, tile_start,
                                    list, list_len, tiles_x, tiles_y, nullptr, image, transmittance,
                                    static_cast<uint32_t *>(ctx->arena), ctx->stream),
            "blend_tiles launch");
    return GSBC_OK;
}

gsbc_status gsbc_blend_tiles_colours(gsbc_ctx *ctx, const float *colours, uint64_t n_prims, const uint32_t *perm,
                                     const float *opacity, const float *footprint, const uint32_t *tile_start,
                                     const uint32_t *list, uint64_t list_len, uint32_t tiles_x, uint32_t tiles_y,
                                     float *image, float *transmittance)
{
    gsbc_status s = begin(ctx);
    if (s) return s;
    ActiveGuard guard(ctx);
    if (!colours || !perm || !opacity || !footprint || !tile_start || !image || (!list && list_len))
        return fail(ctx, GSBC_E_ARG, "NULL pointer argument");
    for (const void *q : {(const void *)colours, (const void *)perm, (const void *)opacity, (const void *)footprint,
                          (const void *)tile_start, (const void *)list, (const void *)image, (const void *)transmittance})
        if (reinterpret_cast<uintptr_t>(q) & 3) return fail(ctx, GSBC_E_ARG, "device arrays must be 4-byte aligned");
    if (n_prims == 0 || n_prims > 0x7FFFFFFFull)
        return fail(ctx, GSBC_E_ARG, "n_prims = %llu not in 1..2^31-1", (unsigned long long)n_prims);
    const uint64_t tiles = (uint64_t)tiles_x * tiles_y;
    if (tiles == 0 || tiles > 0x7FFFFFFFull) return fail(ctx, GSBC_E_ARG, "%u x %u tiles", tiles_x, tiles_y);
    if ((s = ensure_arena(ctx, tiles * sizeof(uint32_t)))) return s;   // the tile schedule
    const float f[3] = {0.0f, 0.0f, 0.0f};   // unused: the colours are given
    HIP_TRY(ctx, launch_blend_tiles(nullptr, BandArgs{}, n_prims, nullptr, perm, f, opacity, footprint, tile_start,
                                    list, list_len, tiles_x, tiles_y, colours, image, transmittance,
                                    static_cast<uint32_t *>(ctx->arena), ctx->stream),
            "blend_tiles launch");
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
