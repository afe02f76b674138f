// rate.hip -- per-band format choice at an exact bit rate (Sec. IV-B: each
// bitstream keeps a fixed block size, so random access survives, while the
// number of bits per primitive is set by which bands use which format).
//
// Band 0 is BC7.  AUTO: of bands 1..S-1, the k with the largest
// coefficient-domain gain (SSE_BC1 - SSE_BC7) * delta^2 are BC7 and the
// rest BC1 (the lower band wins ties); every upgrade costs the same bits,
// so the k largest gains minimise the total error at that budget.
// AUTO_ZERO: each band 1..S-1 is BC7, BC1 or not stored at all (0 bits; its
// coefficients decode to zero), at an exact number of four-bit units, with
// the least total distortion, found by dynamic programming over bands and
// units (the costs 2, 1, 0 are not uniform, so no greedy order is exact).
// Selection and the stream copy run on the device (no host round trip).
#include "gsbc_internal.h"

namespace gsbc {
namespace {

__device__ void layout_streams(const uint32_t fmt[16], uint32_t S, uint64_t nblk, RateSel *sel)
{
    uint64_t pos = 0;
    for (uint32_t q = 0; q < 16; q++) {
        sel->format[q] = q < S ? fmt[q] : 0u;
        sel->offset[q] = q < S ? pos : 0u;
        if (q < S) {
            pos += fmt[q] == GSBC_FMT_NONE ? 0 : nblk * (fmt[q] == GSBC_FMT_BC1 ? 8 : 16);
            pos = (pos + 15) & ~(uint64_t)15;
        }
    }
    sel->payload_bytes = pos;
}

__global__ void k_rate_select(const unsigned long long *sse1, const unsigned long long *sse7, BandArgs b,
                              uint32_t S, uint32_t k, uint64_t nblk, RateSel *sel)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double gain[16];
    for (uint32_t q = 1; q < S; q++) {
        double d = (double)b.delta[q];
        gain[q] = (double)((long long)sse1[q] - (long long)sse7[q]) * (d * d);
    }
    uint32_t fmt[16];
    fmt[0] = GSBC_FMT_BC7;
    for (uint32_t q = 1; q < 16; q++) fmt[q] = GSBC_FMT_BC1;
    for (uint32_t pick = 0; pick < k; pick++) {
        int best = -1;
        for (uint32_t q = 1; q < S; q++) {
            if (fmt[q] == GSBC_FMT_BC7) continue;
            if (best < 0 || gain[q] > gain[best]) best = (int)q;
        }
        fmt[best] = GSBC_FMT_BC7;
    }
    layout_streams(fmt, S, nblk, sel);
}

// Code histogram of every band's R, G and B texel channels: one workgroup
// per (band, slice of blocks), counts in LDS, then added to hist[band][256].
__global__ __launch_bounds__(256) void k_band_hist(const uint8_t *tex, uint64_t nblk,
                                                   unsigned long long *hist)
{
    __shared__ uint32_t h[256];
    const uint32_t band = blockIdx.y;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t *t = reinterpret_cast<const uint32_t *>(tex + (uint64_t)band * nblk * 64);
    const uint64_t words = nblk * 16;   // one RGBA texel per word
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (uint64_t)gridDim.x * 256) {
        const uint32_t w = t[i];
        atomicAdd(&h[w & 255u], 1u);
        atomicAdd(&h[(w >> 8) & 255u], 1u);
        atomicAdd(&h[(w >> 16) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[band * 256 + threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// AUTO_ZERO choice for U units over bands 1..S-1 (BC7 2, BC1 1, none 0).
// Band distortions: SSE * delta^2 for the coded formats; for none, the sum
// over codes q (ascending) of count_q * (vmin + q delta)^2.  least[b][u] is
// the least total of bands b..S-1 with u units, each band's distortion
// added to the total of the later bands (rounded addition is monotone, so
// the least total splits over the choice at band b); the choice then walks
// the bands upward taking, at each, the first of BC7, BC1, none that keeps
// the least total.
__global__ void k_rate_select_zero(const unsigned long long *sse1, const unsigned long long *sse7,
                                   const unsigned long long *hist, BandArgs b, uint32_t S, uint32_t U,
                                   uint64_t nblk, RateSel *sel)
{
    __shared__ double dist[16][3];
    const uint32_t t = threadIdx.x;
    if (t >= 1 && t < S) {   // one lane per band
        const double d = (double)b.delta[t];
        dist[t][0] = (double)sse7[t] * (d * d);
        dist[t][1] = (double)sse1[t] * (d * d);
        double z = 0.0;
        for (int q = 0; q < 256; q++) {
            const double v = (double)b.vmin[t] + (double)q * d;
            z += (double)hist[t * 256 + q] * (v * v);
        }
        dist[t][2] = z;
    }
    __syncthreads();
    if (t != 0) return;
    constexpr int kUnits[3] = {2, 1, 0};
    constexpr uint32_t kCode[3] = {GSBC_FMT_BC7, GSBC_FMT_BC1, GSBC_FMT_NONE};
    double least[17][31];
    bool ok[17][31];
    for (int u = 0; u <= 30; u++) {
        ok[S][u] = u == 0;
        least[S][u] = 0.0;
    }
    for (int band = (int)S - 1; band >= 1; band--)
        for (int u = 0; u <= 30; u++) {
            ok[band][u] = false;
            for (int o = 0; o < 3; o++) {
                const int r = u - kUnits[o];
                if (r < 0 || !ok[band + 1][r]) continue;
                const double v = dist[band][o] + least[band + 1][r];
                if (!ok[band][u] || v < least[band][u]) {
                    least[band][u] = v;
                    ok[band][u] = true;
                }
            }
        }
    uint32_t fmt[16];
    fmt[0] = GSBC_FMT_BC7;
    for (uint32_t q = 1; q < 16; q++) fmt[q] = GSBC_FMT_BC1;
    int u = (int)U;
    for (uint32_t band = 1; band < S; band++)
        for (int o = 0; o < 3; o++) {
            const int r = u - kUnits[o];
            if (r < 0 || !ok[band + 1][r] || dist[band][o] + least[band + 1][r] != least[band][u]) continue;
            fmt[band] = kCode[o];
            u = r;
            break;
        }
    layout_streams(fmt, S, nblk, sel);
}

// blockIdx.y = band; 8-byte words.  A stream with no bits copies nothing.
__global__ __launch_bounds__(256) void k_copy_streams(const uint8_t *src1, const uint64_t *off1,
                                                      const uint8_t *src7, const uint64_t *off7,
                                                      const RateSel *sel, uint64_t nblk, uint8_t *out)
{
    const int q = blockIdx.y;
    if (sel->format[q] == GSBC_FMT_NONE) return;
    const bool bc1 = sel->format[q] == GSBC_FMT_BC1;
    const uint64_t words = nblk * (bc1 ? 1 : 2);
    const uint64_t padded = (words + 1) & ~(uint64_t)1;   // streams are 16-byte aligned
    const uint64_t *src = reinterpret_cast<const uint64_t *>(bc1 ? src1 + off1[q] : src7 + off7[q]);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + sel->offset[q]);
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < padded; w += (uint64_t)gridDim.x * blockDim.x)
        dst[w] = w < words ? src[w] : 0ull;
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_rate_select(const unsigned long long *sse1, const unsigned long long *sse7, const BandArgs &b,
                              uint32_t S, uint32_t k, uint64_t nblk, RateSel *sel, hipStream_t st)
{
    GSBC_LAUNCH("rate_select", k_rate_select, dim3(1), dim3(64), 0, st, sse1, sse7, b, S, k, nblk, sel);
    return hipGetLastError();
}

hipError_t launch_band_hist(const uint8_t *tex, uint32_t S, uint64_t nblk, unsigned long long *hist, hipStream_t st)
{
    uint64_t gx = (nblk * 16 + 255) / 256;
    gx = gx > 256 ? 256 : (gx == 0 ? 1 : gx);
    GSBC_LAUNCH("band_hist", k_band_hist, dim3((uint32_t)gx, S), dim3(256), 0, st, tex, nblk, hist);
    return hipGetLastError();
}

hipError_t launch_rate_select_zero(const unsigned long long *sse1, const unsigned long long *sse7,
                                   const unsigned long long *hist, const BandArgs &b, uint32_t S, uint32_t U,
                                   uint64_t nblk, RateSel *sel, hipStream_t st)
{
    GSBC_LAUNCH("rate_select", k_rate_select_zero, dim3(1), dim3(64), 0, st, sse1, sse7, hist, b, S, U, nblk, sel);
    return hipGetLastError();
}

hipError_t launch_copy_streams(const uint8_t *src1, const uint64_t *off1, const uint8_t *src7,
                               const uint64_t *off7, const RateSel *sel, uint32_t S, uint64_t nblk, uint8_t *out,
                               hipStream_t st)
{
    uint64_t words = nblk * 2;
    uint32_t gx = (uint32_t)((words + 255) / 256);
    gx = gx > 1024 ? 1024 : (gx == 0 ? 1 : gx);
    GSBC_LAUNCH("copy_streams", k_copy_streams, dim3(gx, S), dim3(256), 0, st, src1, off1, src7, off7, sel, nblk, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    GSBC_LAUNCH("fill", k_fill_u64, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace gsbc
