// bc1_encode.hip -- BC1 encoder for gfx950 (BTC with two RGB565 reference
// colours and 2-bit indices, Sec. III-A; the paper codes each 4x4 band block
// this way, Sec. V).
//
// One lane codes one block, so the whole split enumeration of the cluster
// fit runs in wave-uniform order: the split bounds, cluster weights and
// normal-equation determinants are scalar, and each lane only evaluates its
// own numerators, quantised endpoints and SSE.  Per-lane prefix sums of the
// ordered texels live in LDS, one column per lane (conflict-free reads at a
// uniform row).  Every decision is integer; ties take the first candidate in
// the fixed enumeration order.
//
// Steps: constant block -> per-channel endpoint tables; otherwise principal
// axis by integer power iteration, texels ordered by projection, every
// 4-cluster and 3-cluster split fitted by least squares and scored by its
// exact SSE, the best canonicalised and re-indexed, then `refine_steps`
// rounds of +-1 moves of the six endpoint channels.
#include "gsbc_internal.h"
#include "bc_format.h"

#include <vector>

namespace gsbc {
namespace {

constexpr int kBlock = 128;   // lanes per workgroup

// Constant-colour endpoint tables per channel width (0: 5 bits, 1: 6 bits).
struct Bc1Tables {
    uint8_t a4[2][256], b4[2][256], e4[2][256];
    uint8_t a3[2][256], b3[2][256], e3[2][256];
};
__constant__ Bc1Tables kTab;

__host__ __device__ inline int e5(int c) { return (c << 3) | (c >> 2); }
__host__ __device__ inline int e6(int c) { return (c << 2) | (c >> 4); }
__host__ __device__ inline int ew(int c, int wide) { return wide ? e6(c) : e5(c); }

__device__ inline int bitlen(int x) { return 32 - __clz(x); }

// Least code c in [0, 2^w) minimising |E(c)*den - num|, den > 0 (lowest c on
// ties).  E is increasing, so the minimiser is the last code with
// E(c)*den <= num or the one after it; the float estimate lands within one
// code of that one and two integer checks settle it.
__device__ inline int quant_code(int num, int den, float inv, int wide)
{
    const int maxc = wide ? 63 : 31;
    float f = (float)num * inv;                    // ~ num/den * maxc/255
    int c = (int)floorf(f);
    c = c < -1 ? -1 : (c > maxc ? maxc : c);
    if (c >= 0 && __mul24(ew(c, wide), den) > num) c--;
    if (c < maxc && __mul24(ew(c + 1, wide), den) <= num) c++;
    if (c < 0) return 0;
    if (c == maxc) return maxc;
    int d0 = num - __mul24(ew(c, wide), den);
    int d1 = __mul24(ew(c + 1, wide), den) - num;
    return d0 <= d1 ? c : c + 1;
}

__device__ inline uint32_t pack565(int r, int g, int b) { return ((uint32_t)r << 11) | ((uint32_t)g << 5) | (uint32_t)b; }

// Order the pair for the mode (4-colour: c0 > c1, 3-colour: c0 <= c1), then
// give each texel its least-SSE palette entry (lowest index on ties).
__device__ inline uint32_t canon_index(uint32_t &c0, uint32_t &c1, bool four, const int (&x)[16][3],
                                       uint32_t &indices)
{
    if ((four && c0 < c1) || (!four && c0 > c1)) { uint32_t t = c0; c0 = c1; c1 = t; }
    int p[4][3];
    int e0[3], e1[3];
    bc1_expand(c0, e0);
    bc1_expand(c1, e1);
    const bool m4 = c0 > c1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        p[0][c] = e0[c];
        p[1][c] = e1[c];
        if (m4) {
            p[2][c] = (uint32_t)(2 * e0[c] + e1[c] + 1) / 3u;
            p[3][c] = (uint32_t)(e0[c] + 2 * e1[c] + 1) / 3u;
        } else {
            p[2][c] = (e0[c] + e1[c] + 1) >> 1;
            p[3][c] = 0;
        }
    }
    uint32_t sse = 0, idx = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int d0 = x[i][0] - p[k][0], d1 = x[i][1] - p[k][1], d2 = x[i][2] - p[k][2];
            uint32_t d = (uint32_t)(d0 * d0 + d1 * d1 + d2 * d2);
            uint32_t key = (d << 2) | (uint32_t)k;   // d < 2^18: exact order, index breaks ties
            best = key < best ? key : best;
        }
        sse += best >> 2;
        idx |= (best & 3u) << (2 * i);
    }
    indices = idx;
    return sse;
}

__device__ void encode_block(const uint32_t (&t)[16], uint32_t refine_steps, int *sP,
                             uint32_t &w0, uint32_t &w1, uint32_t &sse_out)
{
    int x[16][3];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        x[i][0] = t[i] & 255;
        x[i][1] = (t[i] >> 8) & 255;
        x[i][2] = (t[i] >> 16) & 255;
    }
    bool constant = true;
#pragma unroll
    for (int i = 1; i < 16; i++) constant &= ((t[i] ^ t[0]) & 0xFFFFFFu) == 0;

    uint32_t c0, c1, idx, sse;
    if (constant) {
        int a4[3], b4[3], a3[3], b3[3], err4 = 0, err3 = 0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            int wide = c == 1, v = x[0][c];
            a4[c] = kTab.a4[wide][v]; b4[c] = kTab.b4[wide][v];
            a3[c] = kTab.a3[wide][v]; b3[c] = kTab.b3[wide][v];
            int e4 = kTab.e4[wide][v], e3 = kTab.e3[wide][v];
            err4 += e4 * e4;
            err3 += e3 * e3;
        }
        bool four = err4 <= err3;
        c0 = four ? pack565(a4[0], a4[1], a4[2]) : pack565(a3[0], a3[1], a3[2]);
        c1 = four ? pack565(b4[0], b4[1], b4[2]) : pack565(b3[0], b3[1], b3[2]);
        sse = canon_index(c0, c1, four, x, idx);
        w0 = c0 | (c1 << 16);
        w1 = idx;
        sse_out = sse;
        return;
    }

    // ---- principal axis (integer power iteration, int32 exact)
    int S[3] = {0, 0, 0}, XX[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    int Q = 0;
#pragma unroll
    for (int i = 0; i < 16; i++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            S[a] += x[i][a];
#pragma unroll
            for (int b = a; b < 3; b++) XX[a][b] += x[i][a] * x[i][b];
            Q += x[i][a] * x[i][a];
        }
    int C[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = a; b < 3; b++) { C[a][b] = 16 * XX[a][b] - S[a] * S[b]; C[b][a] = C[a][b]; }
    // row of the largest diagonal entry (lowest index on ties), by selects
    const int j = (C[1][1] > C[0][0]) ? ((C[2][2] > C[1][1]) ? 2 : 1) : ((C[2][2] > C[0][0]) ? 2 : 0);
    const int dmax = j == 0 ? C[0][0] : (j == 1 ? C[1][1] : C[2][2]);
    int tsh = max(0, bitlen(dmax) - 14);
    int Cs[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) Cs[a][b] = C[a][b] >> tsh;
    int v[3];
#pragma unroll
    for (int b = 0; b < 3; b++) v[b] = j == 0 ? Cs[0][b] : (j == 1 ? Cs[1][b] : Cs[2][b]);
#pragma unroll
    for (int it = 0; it < 8; it++) {
        int u[3];
#pragma unroll
        for (int a = 0; a < 3; a++) u[a] = Cs[a][0] * v[0] + Cs[a][1] * v[1] + Cs[a][2] * v[2];
        int m = max(abs(u[0]), max(abs(u[1]), abs(u[2])));
        int s = max(0, bitlen(m) - 15);
#pragma unroll
        for (int a = 0; a < 3; a++) v[a] = u[a] >> s;
    }
    if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;

    // ---- order texels by (projection, index); prefix sums into LDS
    int proj[16];
#pragma unroll
    for (int i = 0; i < 16; i++) proj[i] = v[0] * x[i][0] + v[1] * x[i][1] + v[2] * x[i][2];
    int rank[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        int r = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) r += (proj[k] < proj[i]) || (proj[k] == proj[i] && k < i);
        rank[i] = r;
    }
    // xs[k] = x of the texel with rank k; P[s] = sum of xs[0..s)
    int run[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k <= 16; k++) {
#pragma unroll
        for (int c = 0; c < 3; c++) sP[(k * 3 + c) * kBlock] = run[c];
        if (k < 16) {
#pragma unroll
            for (int i = 0; i < 16; i++)
                if (rank[i] == k) { run[0] += x[i][0]; run[1] += x[i][1]; run[2] += x[i][2]; }
        }
    }
    const int tot[3] = {run[0], run[1], run[2]};

    // ---- cluster fit over every split (4-colour list, then 3-colour list)
    uint32_t best = 0xFFFFFFFFu;
    int bq[6] = {0, 0, 0, 0, 0, 0};
    bool bfour = true;
    for (int list = 0; list < 2; list++) {
        const bool four = list == 0;
        const int F = four ? 3 : 2;
        for (int s1 = 0; s1 <= 16; s1++) {
            for (int s2 = s1; s2 <= 16; s2++) {
                const int s3lo = four ? s2 : 16;
                for (int s3 = s3lo; s3 <= 16; s3++) {
                    int n0 = s1, n1 = s2 - s1, n2 = s3 - s2, n3 = 16 - s3;
                    int A, B, AB;
                    if (four) { A = 9 * n0 + 4 * n1 + n2; B = n1 + 4 * n2 + 9 * n3; AB = 2 * (n1 + n2); }
                    else { A = 4 * n0 + n1; B = n1 + 4 * n2; AB = n1; }
                    int det = A * B - AB * AB;
                    if (det == 0) continue;
                    float inv5 = 31.0f / (255.0f * (float)det), inv6 = 63.0f / (255.0f * (float)det);
                    int q0[3], q1[3];
                    int sse = Q;
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        int P1 = sP[(s1 * 3 + c) * kBlock], P2 = sP[(s2 * 3 + c) * kBlock];
                        int P3 = sP[(s3 * 3 + c) * kBlock];
                        int X0 = P1, X1 = P2 - P1, X2 = P3 - P2, X3 = tot[c] - P3;
                        int SA, SB;
                        if (four) { SA = 3 * X0 + 2 * X1 + X2; SB = X1 + 2 * X2 + 3 * X3; }
                        else { SA = 2 * X0 + X1; SB = X1 + 2 * X2; }
                        int num0 = F * (__mul24(B, SA) - __mul24(AB, SB));
                        int num1 = F * (__mul24(A, SB) - __mul24(AB, SA));
                        const int wide = c == 1;
                        const float inv = wide ? inv6 : inv5;
                        q0[c] = quant_code(num0, det, inv, wide);
                        q1[c] = quant_code(num1, det, inv, wide);
                        int e0 = ew(q0[c], wide), e1 = ew(q1[c], wide);
                        if (four) {
                            int p1 = (uint32_t)(2 * e0 + e1 + 1) / 3u, p2 = (uint32_t)(e0 + 2 * e1 + 1) / 3u;
                            sse += __mul24(n0, e0 * e0) - 2 * __mul24(e0, X0);
                            sse += __mul24(n1, p1 * p1) - 2 * __mul24(p1, X1);
                            sse += __mul24(n2, p2 * p2) - 2 * __mul24(p2, X2);
                            sse += __mul24(n3, e1 * e1) - 2 * __mul24(e1, X3);
                        } else {
                            int p1 = (e0 + e1 + 1) >> 1;
                            sse += __mul24(n0, e0 * e0) - 2 * __mul24(e0, X0);
                            sse += __mul24(n1, p1 * p1) - 2 * __mul24(p1, X1);
                            sse += __mul24(n2, e1 * e1) - 2 * __mul24(e1, X2);
                        }
                    }
                    if ((uint32_t)sse < best) {
                        best = (uint32_t)sse;
                        bq[0] = q0[0]; bq[1] = q0[1]; bq[2] = q0[2];
                        bq[3] = q1[0]; bq[4] = q1[1]; bq[5] = q1[2];
                        bfour = four;
                    }
                }
            }
        }
    }

    c0 = pack565(bq[0], bq[1], bq[2]);
    c1 = pack565(bq[3], bq[4], bq[5]);
    sse = canon_index(c0, c1, bfour, x, idx);

    // ---- refinement: best of the 12 one-step moves, taken if strictly better
    for (uint32_t step = 0; step < refine_steps; step++) {
        const bool four = c0 > c1;
        int cur[6] = {(int)(c0 >> 11) & 31, (int)(c0 >> 5) & 63, (int)c0 & 31,
                      (int)(c1 >> 11) & 31, (int)(c1 >> 5) & 63, (int)c1 & 31};
        uint32_t nb_sse = 0xFFFFFFFFu, nb0 = 0, nb1 = 0, nbi = 0;
#pragma unroll
        for (int q = 0; q < 12; q++) {
            int ch = q >> 1, dlt = (q & 1) ? 1 : -1;
            int maxc = (ch % 3 == 1) ? 63 : 31;
            int cand[6] = {cur[0], cur[1], cur[2], cur[3], cur[4], cur[5]};
            int nv = cand[ch] + dlt;
            cand[ch] = nv < 0 ? 0 : (nv > maxc ? maxc : nv);
            uint32_t a = pack565(cand[0], cand[1], cand[2]), b = pack565(cand[3], cand[4], cand[5]), ii;
            uint32_t s = canon_index(a, b, four, x, ii);
            if (s < nb_sse) { nb_sse = s; nb0 = a; nb1 = b; nbi = ii; }
        }
        if (nb_sse < sse) { sse = nb_sse; c0 = nb0; c1 = nb1; idx = nbi; }
        else break;
    }
    w0 = c0 | (c1 << 16);
    w1 = idx;
    sse_out = sse;
}

__global__ __launch_bounds__(kBlock) void k_bc1_encode(EncodeArgs a)
{
    __shared__ int sP[17 * 3 * kBlock];
    const uint64_t g0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t total = (uint64_t)a.nbands * a.nblk;
    const bool live = g0 < total;
    const uint64_t g = live ? g0 : total - 1;   // past-the-end lanes redo the last block, write nothing
    const uint32_t band = a.band0 + (uint32_t)(g / a.nblk);
    const uint64_t b = g % a.nblk;
    const uint4 *src = reinterpret_cast<const uint4 *>(a.textures + ((uint64_t)band * a.nblk + b) * 64);
    uint32_t t[16];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        uint4 v = src[q];
        t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
    }
    uint32_t w0, w1, sse;
    encode_block(t, a.refine_steps, sP + threadIdx.x, w0, w1, sse);
    if (live) {
        uint2 *dst = reinterpret_cast<uint2 *>(a.out + a.out_offset[band] + b * 8);
        *dst = make_uint2(w0, w1);
        if (b == a.nblk - 1 && (a.nblk & 1)) dst[1] = make_uint2(0, 0);   // 16-byte stream alignment
    }
    if (a.band_sse) band_add(a.band_sse, band, sse, live);
}

// Host-side construction of the constant-colour tables: for each channel
// width and target value, the code pair whose 4-colour 2/3 point (resp.
// 3-colour midpoint) is nearest the target; ties by |a-b|, then a, then b.
void build_tables(Bc1Tables &T)
{
    for (int wide = 0; wide < 2; wide++) {
        const int nc = wide ? 64 : 32;
        for (int mode = 0; mode < 2; mode++) {
            // every pair's value, then the best pair per target
            std::vector<int> val(nc * nc);
            for (int a = 0; a < nc; a++)
                for (int b = 0; b < nc; b++) {
                    int ea = ew(a, wide), eb = ew(b, wide);
                    val[a * nc + b] = mode == 0 ? (2 * ea + eb + 1) / 3 : (ea + eb + 1) >> 1;
                }
            for (int v = 0; v < 256; v++) {
                int best = -1;
                int be = 0, bd = 0;
                for (int pr = 0; pr < nc * nc; pr++) {
                    int a = pr / nc, b = pr % nc;
                    int e = val[pr] > v ? val[pr] - v : v - val[pr];
                    int d = a > b ? a - b : b - a;
                    // pairs are visited in (a, b) order, so strict comparisons keep the lowest
                    if (best < 0 || e < be || (e == be && d < bd)) { best = pr; be = e; bd = d; }
                }
                uint8_t *A = mode == 0 ? T.a4[wide] : T.a3[wide];
                uint8_t *B = mode == 0 ? T.b4[wide] : T.b3[wide];
                uint8_t *E = mode == 0 ? T.e4[wide] : T.e3[wide];
                A[v] = (uint8_t)(best / nc);
                B[v] = (uint8_t)(best % nc);
                E[v] = (uint8_t)be;
            }
        }
    }
}

}  // namespace

hipError_t upload_bc1_tables(hipStream_t st)
{
    static Bc1Tables host;
    static bool built = false;
    if (!built) { build_tables(host); built = true; }
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(kTab), &host, sizeof(host), 0, hipMemcpyHostToDevice, st);
}

hipError_t launch_bc1_encode(const EncodeArgs &a, hipStream_t st)
{
    uint64_t total = (uint64_t)a.nbands * a.nblk;
    if (total == 0) return hipSuccess;
    GSBC_LAUNCH("bc1_encode", k_bc1_encode, dim3((uint32_t)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace gsbc
