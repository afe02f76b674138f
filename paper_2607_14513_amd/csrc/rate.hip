// rate.hip -- per-band format choice at an exact bit rate (Sec. IV-B: each
// bitstream keeps a fixed block size, so random access survives, while the
// number of bits per primitive is set by which bands use the larger format).
//
// Band 0 is BC7.  Of bands 1..15, the k with the largest coefficient-domain
// gain (SSE_BC1 - SSE_BC7) * delta^2 are BC7 and the rest BC1 (the lower
// band wins ties).  Every upgrade costs the same number of bits, so taking
// the k largest gains minimises the total coefficient error at that budget.
// Selection and the stream copy run on the device (no host round trip).
#include "gsbc_internal.h"

namespace gsbc {
namespace {

__global__ void k_rate_select(const unsigned long long *sse1, const unsigned long long *sse7, BandArgs b,
                              uint32_t k, uint64_t nblk, RateSel *sel)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double gain[16];
    for (int q = 1; q < 16; q++) {
        double d = (double)b.delta[q];
        gain[q] = (double)((long long)sse1[q] - (long long)sse7[q]) * (d * d);
    }
    uint32_t fmt[16];
    fmt[0] = 7;
    for (int q = 1; q < 16; q++) fmt[q] = 1;
    for (uint32_t pick = 0; pick < k; pick++) {
        int best = -1;
        for (int q = 1; q < 16; q++) {
            if (fmt[q] == 7) continue;
            if (best < 0 || gain[q] > gain[best]) best = q;
        }
        fmt[best] = 7;
    }
    uint64_t pos = 0;
    for (int q = 0; q < 16; q++) {
        sel->format[q] = fmt[q];
        sel->offset[q] = pos;
        pos += nblk * (fmt[q] == 1 ? 8 : 16);
        pos = (pos + 15) & ~(uint64_t)15;
    }
    sel->payload_bytes = pos;
}

// blockIdx.y = band; 8-byte words.
__global__ __launch_bounds__(256) void k_copy_streams(const uint8_t *src1, const uint64_t *off1,
                                                      const uint8_t *src7, const uint64_t *off7,
                                                      const RateSel *sel, uint64_t nblk, uint8_t *out)
{
    const int q = blockIdx.y;
    const bool bc1 = sel->format[q] == 1;
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
                              uint32_t k, uint64_t nblk, RateSel *sel, hipStream_t st)
{
    GSBC_LAUNCH("rate_select", k_rate_select, dim3(1), dim3(64), 0, st, sse1, sse7, b, k, nblk, sel);
    return hipGetLastError();
}

hipError_t launch_copy_streams(const uint8_t *src1, const uint64_t *off1, const uint8_t *src7,
                               const uint64_t *off7, const RateSel *sel, uint64_t nblk, uint8_t *out,
                               hipStream_t st)
{
    uint64_t words = nblk * 2;
    uint32_t gx = (uint32_t)((words + 255) / 256);
    gx = gx > 1024 ? 1024 : (gx == 0 ? 1 : gx);
    GSBC_LAUNCH("copy_streams", k_copy_streams, dim3(gx, 16), dim3(256), 0, st, src1, off1, src7, off7, sel, nblk, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    GSBC_LAUNCH("fill", k_fill_u64, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace gsbc
