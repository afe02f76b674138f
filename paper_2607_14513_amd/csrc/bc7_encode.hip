// bc7_encode.hip -- BC7 encoder for gfx950 (BTC with 1-3 reference-colour
// pairs per block, Sec. III-B; the paper codes 4x4 band blocks this way,
// Sec. V).
//
// Search: 285 candidates in a fixed order (mode 0 partitions 0..15; modes
// 1, 2, 3 partitions 0..63; mode 4 rotation x index-selection; mode 5
// rotation; mode 6; mode 7 partitions 0..63).  Each subset is fitted on its
// own: identical texels use precomputed single-value endpoint tables;
// otherwise the endpoints are the texels of least and greatest projection on
// the principal axis (integer power iteration), quantised for every p-bit
// choice, texels take their least-SSE palette entry, and one least-squares
// refit is kept if it lowers the SSE.  The winner minimises
// (SSE << 9) | candidate, a total order, so the result is independent of how
// candidates are spread over lanes.
//
// Layout on the GPU: one lane per block, all lanes of a wave walk the
// candidates in the same order, so partition masks, anchors and mode
// parameters are wave-uniform (scalar registers) and only the texel
// arithmetic is per lane.  Pass 1 keeps only the best key; pass 2 re-fits
// each lane's winner (identical arithmetic) to emit its bits.
#include "gsbc_internal.h"
#include "bc_format.h"

#include <mutex>
#include <vector>

namespace gsbc {

// Zero, read from memory (external linkage, so it is not folded): see
// entry_const.
__constant__ uint32_t g_bc7_opaque_zero = 0u;

namespace {

// ---- tables (device global memory, built on the host at first use)
// nearest[cls][p][t]: code c minimising |value(c, p) - t| (lowest on ties)
// in the low byte, value(c, p) in the high byte; cls = (cb - 4) * 2 + has_pbit.
// near64[cls][p][t]: 64 value(c, p) of the same code (the search reads only
// values, in the scale its palette entries use).
// sv[cls][p0 + 2 p1][slot][v]: single-value pair (c0 | c1 << 8 | err << 16)
// whose interpolation at weight(nb, K) is nearest v; slot = nb offset + K.
struct Tables {
    const uint16_t *nearest;
    const uint16_t *near64;
    const uint32_t *sv;
};
constexpr int kSlots = 28;
__host__ __device__ constexpr int slot_of(int nb, int k) { return (nb == 2 ? 0 : nb == 3 ? 4 : 12) + k; }
__host__ __device__ constexpr int cls_of(int cb, int pb) { return (cb - 4) * 2 + (pb ? 1 : 0); }

__host__ __device__ constexpr int ep_value(int code, int p, int cb, int pb)
{
    return pb ? expand_bits((code << 1) | p, cb + 1) : expand_bits(code, cb);
}

__device__ __forceinline__ int bitlen(int x) { return 32 - __clz(x); }

// ---- candidate geometry
__device__ __forceinline__ uint32_t mask3(int p, int s)
{
    uint32_t w = kPart3[p], m = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) m |= (((w >> (2 * i)) & 3) == (uint32_t)s ? 1u : 0u) << i;
    return m;
}
__device__ __forceinline__ uint32_t mask2(int p, int s)
{
    uint32_t w = kPart2[p];
    return s ? w : (~w & 0xFFFFu);
}

// Candidate index -> (mode, partition, rotation, index selection)
__device__ __forceinline__ void candidate(int ci, int &m, int &p, int &r, int &s)
{
    p = r = s = 0;
    if (ci < 16) { m = 0; p = ci; }
    else if (ci < 80) { m = 1; p = ci - 16; }
    else if (ci < 144) { m = 2; p = ci - 80; }
    else if (ci < 208) { m = 3; p = ci - 144; }
    else if (ci < 216) { m = 4; r = (ci - 208) >> 1; s = (ci - 208) & 1; }
    else if (ci < 220) { m = 5; r = ci - 216; }
    else if (ci < 221) { m = 6; }
    else { m = 7; p = ci - 221; }
}

// ---- texels in LDS
//
// Texels sit in LDS, one column per lane, scaled by -8: rg holds -8 R and
// -8 G as 16-bit halves, bx holds -8 B.  Because |x|^2 is the same for every
// palette entry, the least-SSE entry is the least 256 (|p|^2 - 2 x.p) + k.
// Each entry is held as E = (64 pR, 64 pG) in 16-bit halves, Eb = 64 pB and
// C = 256 |p|^2 + k, so one texel x entry evaluation is
//   t = (-8 B) * Eb + C                    (v_mad_i32_i24)
//   t = (-8 R, -8 G) . E + t               (v_dot2c_i32_i16)
//   best = min(best, t)                    (half a v_min3_i32)
// and the members' minima plus 256 sum |x|^2 (taken once per subset from
// its sums) give 256 SSE + sum k exactly (all terms stay within int32:
// |t| < 2^27).  Summed over at most 16 members the k terms stay below 256,
// so the subset SSE is the sum shifted right by 8.  The 64-scaled entries
// are what the interpolation (64 - w) e0 + w e1 + 32 yields once its low six
// bits are masked off, which keeps palette construction short.
// In the search the subset masks are wave-uniform, so texel loops walk the
// set bits of a mask with scalar control.
constexpr int kWG = 256;
constexpr int kQEntries = 10 * 2 * 256;
constexpr int kScaleNeg = -8;          // texel scale in LDS

struct TexLds {
    uint32_t rg[16][kWG];
    int32_t bx[16][kWG];
    uint16_t q[kQEntries];        // search: near64; emit: nearest
};

typedef short short2_t __attribute__((ext_vector_type(2)));

// -8 times the value 255 (a rotated-out channel's replacement)
constexpr int kNeg255 = kScaleNeg * 255;

// Texel i of this lane in the LDS layout; rotation r puts 255 in channel r-1.
__device__ __forceinline__ void texel(const TexLds &S, int i, int rot, uint32_t &rg, int &b)
{
    rg = S.rg[i][threadIdx.x];
    b = S.bx[i][threadIdx.x];
    if (rot) {
        if (rot == 1) rg = (rg & 0xFFFF0000u) | ((uint32_t)kNeg255 & 0xFFFFu);
        else if (rot == 2) rg = (rg & 0xFFFFu) | ((uint32_t)kNeg255 << 16);
        else b = kNeg255;
    }
}

// The texel's channels, negated: (-R, -G, -B) (exact: the stored values are
// multiples of 8).
__device__ __forceinline__ void unpack_neg(uint32_t rg, int b, int (&x)[3])
{
    x[0] = __builtin_amdgcn_sbfe((int)rg, 3, 13);
    x[1] = (int)rg >> 19;
    x[2] = b >> 3;
}

__device__ __forceinline__ void unpack(uint32_t rg, int b, int (&x)[3])
{
    unpack_neg(rg, b, x);
    x[0] = -x[0];
    x[1] = -x[1];
    x[2] = -x[2];
}

// Per-subset data shared across modes: whether every member is the same
// colour, and the two endpoint colours (texels of least and greatest
// projection on the principal axis, or the common colour).
struct Prep {
    bool same;
    int lo[3], hi[3];
    int nSx[3];  // negated member sums per channel (for the least-squares refit)
    int xx;      // sum of |x|^2 over the members
};

// Member sums of a subset: count, negated per-channel sums and the six
// distinct products (RR, RG, RB, GG, GB, BB; the same for negated values).
// Integer, so the sums of disjoint subsets add up exactly: the last subset
// of a partition is the block total minus the others.
struct Sums {
    int n;
    int nSx[3];
    int XX[6];
};

__device__ __forceinline__ Sums subset_sums(const TexLds &S, uint32_t mask, int rot)
{
    Sums m;
    m.n = __popc(mask);
    m.nSx[0] = m.nSx[1] = m.nSx[2] = 0;
#pragma unroll
    for (int q = 0; q < 6; q++) m.XX[q] = 0;
    // -8 R and -8 G summed in the 16-bit halves of one word (at most 16
    // members: |sum| <= 32640)
    short2_t srg = {0, 0};
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
        uint32_t rg;
        int b;
        texel(S, __ffs(mm) - 1, rot, rg, b);
        int x[3];
        unpack_neg(rg, b, x);
        srg += __builtin_bit_cast(short2_t, rg);
        m.nSx[2] += x[2];
        m.XX[0] += mul_i24(x[0], x[0]); m.XX[1] += mul_i24(x[0], x[1]); m.XX[2] += mul_i24(x[0], x[2]);
        m.XX[3] += mul_i24(x[1], x[1]); m.XX[4] += mul_i24(x[1], x[2]); m.XX[5] += mul_i24(x[2], x[2]);
    }
    m.nSx[0] = (int)srg.x >> 3;
    m.nSx[1] = (int)srg.y >> 3;
    return m;
}

__device__ __forceinline__ Sums sums_minus(const Sums &t, const Sums &a)
{
    Sums m;
    m.n = t.n - a.n;
#pragma unroll
    for (int c = 0; c < 3; c++) m.nSx[c] = t.nSx[c] - a.nSx[c];
#pragma unroll
    for (int q = 0; q < 6; q++) m.XX[q] = t.XX[q] - a.XX[q];
    return m;
}

// Principal axis and endpoint texels of a subset from its sums.  The exact
// covariance C = n XX - Sx Sx^T (the same from negated sums) is zero exactly
// when every member has the same colour.
__device__ __forceinline__ Prep prep_subset(const TexLds &S, uint32_t mask, int rot, const Sums &m)
{
    Prep P;
    // n <= 16, XX < 2^21 and |Sx| < 2^12: 24-bit multiplies with exact products
    const int n = m.n;
    int C[3][3];
    C[0][0] = __mul24(n, m.XX[0]) - __mul24(m.nSx[0], m.nSx[0]);
    C[0][1] = C[1][0] = __mul24(n, m.XX[1]) - __mul24(m.nSx[0], m.nSx[1]);
    C[0][2] = C[2][0] = __mul24(n, m.XX[2]) - __mul24(m.nSx[0], m.nSx[2]);
    C[1][1] = __mul24(n, m.XX[3]) - __mul24(m.nSx[1], m.nSx[1]);
    C[1][2] = C[2][1] = __mul24(n, m.XX[4]) - __mul24(m.nSx[1], m.nSx[2]);
    C[2][2] = __mul24(n, m.XX[5]) - __mul24(m.nSx[2], m.nSx[2]);
    P.same = (C[0][0] | C[1][1] | C[2][2]) == 0;
    P.nSx[0] = m.nSx[0]; P.nSx[1] = m.nSx[1]; P.nSx[2] = m.nSx[2];
    P.xx = m.XX[0] + m.XX[3] + m.XX[5];
    if (P.same) {
        uint32_t rg;
        int b;
        texel(S, __ffs(mask) - 1, rot, rg, b);
        unpack(rg, b, P.lo);
        P.hi[0] = P.lo[0]; P.hi[1] = P.lo[1]; P.hi[2] = P.lo[2];
        return P;
    }
    // principal axis: integer power iteration on the exact covariance
    // row of the largest diagonal entry (lowest index on ties), by selects
    const int j = (C[1][1] > C[0][0]) ? ((C[2][2] > C[1][1]) ? 2 : 1) : ((C[2][2] > C[0][0]) ? 2 : 0);
    const int tsh = max(0, bitlen(j == 0 ? C[0][0] : (j == 1 ? C[1][1] : C[2][2])) - 14);
    int Cs[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) Cs[a][c] = C[a][c] >> tsh;
    int v[3];
#pragma unroll
    for (int c = 0; c < 3; c++) v[c] = j == 0 ? Cs[0][c] : (j == 1 ? Cs[1][c] : Cs[2][c]);
    // |Cs| <= 2^14 (the largest diagonal is below 2^14 and bounds every entry
    // of the positive semi-definite C) and |v| <= 2^15, so the products are
    // 16-bit dot products with exact 32-bit sums (|u| < 3 * 2^29).
    short2_t c01[3];
#pragma unroll
    for (int a = 0; a < 3; a++) c01[a] = short2_t{(short)Cs[a][0], (short)Cs[a][1]};
#pragma unroll
    for (int it = 0; it < 8; it++) {
        const short2_t v01 = {(short)v[0], (short)v[1]};
        int u[3];
        // the third term as a 24-bit product (|Cs| <= 2^14, |v| <= 2^15)
        // accumulated into by the dot product of the first two
#pragma unroll
        for (int a = 0; a < 3; a++) u[a] = __builtin_amdgcn_sdot2(c01[a], v01, __mul24(Cs[a][2], v[2]), false);
        // max(max |u_a|, 1) as max(max u, -min u, 1): its bit length minus 15,
        // at least 0, is the shift that brings max |v| below 2^15
        const int mx = max(max(u[0], max(u[1], u[2])), max(-min(u[0], min(u[1], u[2])), 1));
        const uint32_t sh = __builtin_elementwise_sub_sat(17u, (uint32_t)__builtin_clz((uint32_t)mx));
#pragma unroll
        for (int a = 0; a < 3; a++) v[a] = u[a] >> sh;
    }
    if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;
    // members of least and greatest projection p, the first of each on ties.
    // The stored texels give q = -8 p in one dot product and one multiply-add
    // (|q| < 2^28); 2 q = -16 p leaves four low bits for the member index:
    // the largest 2q + 15 - i is the least p (first i), the least 2q + i is
    // the greatest p (first i).
    const short2_t v01 = {(short)v[0], (short)v[1]};
    int klo = (int)0x80000000, khi = 0x7FFFFFFF;
    for (uint32_t mm = mask; mm; mm &= mm - 1) {
        const int i = __ffs(mm) - 1;
        uint32_t rg;
        int b;
        texel(S, i, rot, rg, b);
        const int q = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, rg), v01, mul_i24(b, v[2]), false);
        klo = max(klo, 2 * q + (15 - i));
        khi = min(khi, 2 * q + i);
    }
    uint32_t rg;
    int b;
    texel(S, 15 - (klo & 15), rot, rg, b);
    unpack(rg, b, P.lo);
    texel(S, khi & 15, rot, rg, b);
    unpack(rg, b, P.hi);
    return P;
}

__device__ __forceinline__ Prep prep_subset(const TexLds &S, uint32_t mask, int rot)
{
    return prep_subset(S, mask, rot, subset_sums(S, mask, rot));
}

// Result of fitting one endpoint pair to a subset.  eval_pair leaves idx in
// member order (IW bits per member, first member lowest; IW = 2 for 2-bit
// indices, else 4); fit_colour returns it by texel position (4 bits at 4 i
// for member i).
struct PairFit {
    uint32_t sse;
    uint64_t idx;
    uint32_t c0, c1;   // endpoint codes, 8 bits per channel, R lowest
    int p0, p1;
};

template <int NB>
constexpr int idx_width() { return NB == 2 ? 2 : 4; }

// Zero, read from memory: added to a constant whose low bits the compiler
// can prove clear of the product it joins, it keeps the sum an addition, so
// product and sum fuse into one v_mad_u32_u24 instead of a multiply and an or.

// Palette entry constant C = 256 |p|^2 + k from the 64-scaled entry:
// (64 p) . (64 p) + 16 k = 16 C, exactly.  The opaque zero keeps 16 k an
// addition (its bits are provably clear of the product's, which would turn
// it into an or), so product and sum fuse into one v_mad_u32_u24.
__device__ __forceinline__ int entry_const(uint32_t e, int eb, int k)
{
    const short2_t es = __builtin_bit_cast(short2_t, e);
    const uint32_t b2k = mul_u24((uint32_t)eb, (uint32_t)eb) + (16u * (uint32_t)k + g_bc7_opaque_zero);
    return __builtin_amdgcn_sdot2(es, es, (int)b2k, false) >> 4;
}

// (c) for one endpoint pair: quantise for every p-bit combination, index
// every member by least SSE; keep the best combination (lowest on ties).
// Up to 32 palette entries are held at once, so each member is read once
// for all combinations (once per combination for 16-entry palettes).  Per
// member and combination the running sum takes 256 SSE + k in one add and
// the index enters a shift register (newest member at the top; it holds the
// n indices in its top IW n bits).  IDX = false: the SSE only.  CODES: the
// LDS table holds code | value << 8 (the emit pass, which needs the codes);
// otherwise it holds 64 value (the search).
template <int CB, int PB, int NB, bool IDX, bool CODES>
__device__ __forceinline__ PairFit eval_pair(const TexLds &S, uint32_t mask, int rot, const int (&lo)[3],
                                             const int (&hi)[3], int xx)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int NE = 1 << NB;
    constexpr int CPV = NPC * NE <= 32 ? NPC : 1;   // combinations per member visit
    constexpr int NP = PB ? 2 : 1;                  // p-bit values of an endpoint
    constexpr int IW = idx_width<NB>();
    constexpr bool WIDE = IW * 16 > 32;             // the indices need two words
    constexpr int cls = cls_of(CB, PB);
    const int n = __popc(mask);
    // each endpoint quantised for each p-bit value: E = (64 v_R, 64 v_G),
    // Eb = 64 v_B, and the codes (emit)
    uint32_t E[2][NP], code[2][NP];
    int Eb[2][NP];
#pragma unroll
    for (int end = 0; end < 2; end++)
#pragma unroll
        for (int p = 0; p < NP; p++) {
            const uint16_t *t = S.q + (cls * 2 + p) * 256;
            const int *v = end ? hi : lo;
            uint32_t e[3];
#pragma unroll
            for (int c = 0; c < 3; c++) e[c] = t[v[c]];
            if (CODES) {
                code[end][p] = (e[0] & 255u) | (e[1] & 255u) << 8 | (e[2] & 255u) << 16;
#pragma unroll
                for (int c = 0; c < 3; c++) e[c] = (e[c] >> 8) << 6;
            } else {
                code[end][p] = 0;
            }
            E[end][p] = e[0] | (e[1] << 16);
            Eb[end][p] = (int)e[2];
        }
    PairFit best;
    best.sse = 0xFFFFFFFFu;
    best.idx = 0;
    best.c0 = best.c1 = 0;
    best.p0 = best.p1 = 0;
#pragma unroll
    for (int pc0 = 0; pc0 < NPC; pc0 += CPV) {
        // Interpolation (64 - w) e0 + w e1 + 32 = (64 e0 + 32) + w (e1 - e0)
        // stays within [32, 16352], so R and G are interpolated together in
        // 16-bit lanes; masking its low six bits gives the 64-scaled entry.
        uint32_t prg[CPV][NE];
        int pb[CPV][NE], pk[CPV][NE];
#pragma unroll
        for (int j = 0; j < CPV; j++) {
            const int pc = pc0 + j;
            const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
            const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
            const uint32_t E0 = E[0][p0], E1 = E[1][p1];
            const int B0 = Eb[0][p0], B1 = Eb[1][p1];
            const short2_t a_rg = __builtin_bit_cast(short2_t, E0 | 0x00200020u);
            const short2_t s_rg = (__builtin_bit_cast(short2_t, E1) - __builtin_bit_cast(short2_t, E0)) >> (short)6;
            const int a_b = B0 | 32, s_b = (B1 - B0) >> 6;
#pragma unroll
            for (int k = 0; k < NE; k++) {
                // entries 0 and NE-1 are the endpoints themselves (weights 0 and 64)
                const short w = (short)bc7_weight(NB, k);
                const uint32_t e = k == 0 ? E0 : k == NE - 1 ? E1
                                 : __builtin_bit_cast(uint32_t, a_rg + s_rg * w) & 0xFFC0FFC0u;
                const int eb = k == 0 ? B0 : k == NE - 1 ? B1 : (a_b + mul_i24(s_b, w)) & ~63;
                prg[j][k] = e;
                pb[j][k] = eb;
                pk[j][k] = entry_const(e, eb, k);
            }
        }
        // 256 SSE + k summed over members: 256 |x|^2 added once per subset
        uint32_t acc[CPV], rlo[CPV], rhi[CPV];
#pragma unroll
        for (int j = 0; j < CPV; j++) {
            acc[j] = 256u * (uint32_t)xx;
            rlo[j] = rhi[j] = 0;
        }
        // least key of one member against combination j's entries
        auto least = [&](uint32_t rg, int b, int j) {
            int kb = 0x7FFFFFFF;
#pragma unroll
            for (int k = 0; k < NE; k++) {
                // with a p-bit per endpoint, entry 0 depends only on p0 and
                // entry NE-1 only on p1: combinations share those keys
                const int js = (PB == 2 && CPV == 4) ? (k == 0 ? (j & 1) : k == NE - 1 ? (j & 2) : j) : j;
                const int key = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, rg),
                                                       __builtin_bit_cast(short2_t, prg[js][k]),
                                                       mul_i24(b, pb[js][k]) + pk[js][k], false);
                kb = min(kb, key);
            }
            return (uint32_t)kb;   // 256 (SSE - |x|^2) + k of this member
        };
        auto push_index = [&](int j, uint32_t kb) {
            if (IDX) {
                if (WIDE) {
                    rlo[j] = __builtin_amdgcn_alignbit(rhi[j], rlo[j], IW);
                    rhi[j] = __builtin_amdgcn_alignbit(kb, rhi[j], IW);
                } else {
                    rlo[j] = __builtin_amdgcn_alignbit(kb, rlo[j], IW);
                }
            }
        };
        // members two at a time (their keys join the sums in one three-way
        // add), then the odd one
        uint32_t m = mask;
        for (; m & (m - 1); m &= m - 1, m &= m - 1) {
            uint32_t rg0, rg1;
            int b0, b1;
            texel(S, __ffs(m) - 1, rot, rg0, b0);
            texel(S, __ffs(m & (m - 1)) - 1, rot, rg1, b1);
#pragma unroll
            for (int j = 0; j < CPV; j++) {
                const uint32_t k0 = least(rg0, b0, j), k1 = least(rg1, b1, j);
                acc[j] += k0 + k1;
                push_index(j, k0);
                push_index(j, k1);
            }
        }
        if (m) {
            uint32_t rg;
            int b;
            texel(S, __ffs(m) - 1, rot, rg, b);
#pragma unroll
            for (int j = 0; j < CPV; j++) {
                const uint32_t kb = least(rg, b, j);
                acc[j] += kb;
                push_index(j, kb);
            }
        }
#pragma unroll
        for (int j = 0; j < CPV; j++) {
            const uint32_t sse = acc[j] >> 8;
            if (sse < best.sse) {
                const int pc = pc0 + j;
                const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
                const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
                best.sse = sse;
                best.idx = !IDX ? 0
                         : WIDE ? (((uint64_t)rhi[j] << 32) | rlo[j]) >> (64 - IW * n)
                                : (uint64_t)(rlo[j] >> (32 - IW * n));
                best.c0 = code[0][p0];
                best.c1 = code[1][p1];
                best.p0 = p0;
                best.p1 = p1;
            }
        }
    }
    return best;
}

// Index weight of NB-bit index k from the weight table packed in bytes
// (v_perm_b32 picks byte k; selector 0x0C gives zero bytes).
__host__ __device__ constexpr uint32_t pack_weights(int nb, int first)
{
    return (uint32_t)bc7_weight(nb, first) | ((uint32_t)bc7_weight(nb, first + 1) << 8) |
           ((uint32_t)bc7_weight(nb, first + 2) << 16) | ((uint32_t)bc7_weight(nb, first + 3) << 24);
}
static_assert(pack_weights(2, 0) == 0x402B1500u && pack_weights(3, 0) == 0x1B120900u &&
              pack_weights(3, 4) == 0x40372E25u, "BC7 weight tables");

// Weight of the index in the low bits of f (the bits above are ignored).
template <int NB>
__device__ __forceinline__ int weight_of(uint32_t f)
{
    const uint32_t sel = (f & (NB == 2 ? 3u : 7u)) | 0x0C0C0C00u;
    if (NB == 2) return (int)__builtin_amdgcn_perm(0u, pack_weights(2, 0), sel);
    if (NB == 3) return (int)__builtin_amdgcn_perm(pack_weights(3, 4), pack_weights(3, 0), sel);
    return bc7_weight(NB, (int)(f & 15u));
}

// (d) least-squares endpoints for the chosen indices; false if singular.
// With weights (64 - w, w) the normal-equation sums follow from the member
// count n, sum(w), sum(w^2), the channel sums Sx and sum(w x):
//   A = 4096 n - 128 sum(w) + sum(w^2), B = sum(w^2), AB = 64 sum(w) - sum(w^2),
//   SA = 64 Sx - SB.
// The sums of w x are taken on the stored texels, -8 x, by 16-bit dot
// products with (w, 0) and (0, w), so every channel sum carries the factor
// -8; the right-hand sides are formed at that scale and the factor is taken
// out exactly (a power of two) with the reciprocal.
template <int NB>
__device__ __forceinline__ bool ls_endpoints(const TexLds &S, uint32_t mask, int rot, uint64_t idx, const int (&nSx)[3],
                                             int (&lo)[3], int (&hi)[3])
{
    constexpr int IW = idx_width<NB>();
    int W1 = 0, W2 = 0, SB8[3] = {0, 0, 0};   // SB8 = -8 sum(w x)
    uint32_t cur = (uint32_t)idx;
    int j = 0;
    for (uint32_t m = mask; m; m &= m - 1, j++) {
        if (IW == 4 && j == 8) cur = (uint32_t)(idx >> 32);
        uint32_t rg;
        int b;
        texel(S, __ffs(m) - 1, rot, rg, b);
        const int w = weight_of<NB>(cur);   // member order
        cur >>= IW;
        W1 += w;
        W2 += (int)mul_u24((uint32_t)w, (uint32_t)w);
        SB8[0] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, rg), __builtin_bit_cast(short2_t, (uint32_t)w),
                                        SB8[0], false);
        SB8[1] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, rg),
                                        __builtin_bit_cast(short2_t, (uint32_t)w << 16), SB8[1], false);
        SB8[2] += mul_i24(b, w);
    }
    const int n = __popc(mask);
    const int A = 4096 * n - 128 * W1 + W2, B = W2, AB = 64 * W1 - W2;
    const double det = fma((double)A, (double)B, -((double)AB * (double)AB));
    if (det == 0.0) return false;
    // 1/det in FP64 from the FP32 reciprocal and two Newton steps (within
    // 2^-50), times 64 (exact) for the numerators' common factor and -1/8
    // (exact) for the texel scale
    double inv = (double)__builtin_amdgcn_rcpf((float)det);
    inv = fma(fma(-det, inv, 1.0), inv, inv);
    inv = -8.0 * fma(fma(-det, inv, 1.0), inv, inv);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        // Exact numerators n = 64 m (|m| < 2^36), here formed as -8 m
        // (|8 m| < 2^39, products and differences exact in FP64).
        // floor(n/det + 1/2) is taken as floor(m * 64 inv + 1/2 + 2^-37):
        // (2 n + det) / (2 det) is a multiple of 1/(2 det) >= 2^-33, and for
        // |n/det| <= 512 the FP64 error is below 2^-40, so the margin never
        // moves the floor; larger quotients clamp to 0 or 255 either way.
        const double SA8 = (double)(512 * nSx[c] - SB8[c]);
        const double m0 = fma((double)B, SA8, -((double)AB * (double)SB8[c]));
        const double m1 = fma((double)A, (double)SB8[c], -((double)AB * SA8));
        // floor then clamp to [0, 255] equals clamp then truncate
        const double q0 = fma(m0, inv, 0.5 + 0x1p-37), q1 = fma(m1, inv, 0.5 + 0x1p-37);
        lo[c] = (int)fmin(fmax(q0, 0.0), 255.0);
        hi[c] = (int)fmin(fmax(q1, 0.0), 255.0);
    }
    return true;
}

// Fit one colour subset with endpoint precision (CB, PB) and NB-bit indices.
// SEARCH: only the SSE is wanted (the search pass, whose LDS table holds 64-
// scaled values); the refit's indices and the positional index layout are
// skipped.
template <int CB, int PB, int NB, bool SEARCH = false>
__device__ __forceinline__ PairFit fit_colour(const TexLds &S, uint32_t mask, int rot, const Prep &P,
                                              const uint32_t *sv)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int cls = cls_of(CB, PB);
    constexpr int IW = idx_width<NB>();
    if (P.same) {
        // (a) single value: best (p-bits, index) from the per-channel tables
        PairFit f;
        f.sse = 0xFFFFFFFFu;
        f.idx = 0;
        f.c0 = f.c1 = 0;
        f.p0 = f.p1 = 0;
        for (int pc = 0; pc < NPC; pc++) {
            const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
            const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
            for (int k = 0; k < (1 << NB); k++) {
                const uint32_t *row = sv + ((uint64_t)(cls * 4 + p0 + 2 * p1) * kSlots + slot_of(NB, k)) * 256;
                uint32_t e = 0, c0 = 0, c1 = 0;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const uint32_t ent = row[P.lo[c]];
                    const uint32_t er = ent >> 16;
                    e += er * er;
                    c0 |= (ent & 255u) << (8 * c);
                    c1 |= ((ent >> 8) & 255u) << (8 * c);
                }
                if (e < f.sse) {
                    f.sse = e;
                    f.idx = (uint64_t)k * 0x1111111111111111ull;
                    f.c0 = c0;
                    f.c1 = c1;
                    f.p0 = p0;
                    f.p1 = p1;
                }
            }
        }
        f.sse *= (uint32_t)__popc(mask);
        return f;
    }
    // (b) endpoints from the principal axis, (c) quantise and index,
    // (d) one least-squares refit kept only if strictly better
    PairFit f = eval_pair<CB, PB, NB, true, !SEARCH>(S, mask, rot, P.lo, P.hi, P.xx);
    int rlo[3], rhi[3];
    if (ls_endpoints<NB>(S, mask, rot, f.idx, P.nSx, rlo, rhi)) {
        PairFit g = eval_pair<CB, PB, NB, !SEARCH, !SEARCH>(S, mask, rot, rlo, rhi, P.xx);
        if (g.sse < f.sse) f = g;
    }
    if (SEARCH) return f;
    // member order -> texel positions
    uint64_t pos = 0, c = f.idx;
    for (uint32_t m = mask; m; m &= m - 1) {
        pos |= (c & ((1u << IW) - 1)) << (4 * (__ffs(m) - 1));
        c >>= IW;
    }
    f.idx = pos;
    return f;
}

// Scalar channel of modes 4 and 5: the 16 values of channel r-1 (rotation
// r > 0) or the constant 255 (r = 0); precision AB bits, NB-bit indices.
// The values are taken negated from the stored texels; every sum below is
// negated with them and the keys are unchanged.
template <int AB, int NB, bool CODES>
__device__ __forceinline__ PairFit fit_scalar(const TexLds &S, int rot, const uint32_t *sv)
{
    constexpr int cls = cls_of(AB, 0);
    auto nvalue = [&](int i) {
        const uint32_t rg = S.rg[i][threadIdx.x];
        const int b = S.bx[i][threadIdx.x];
        return rot == 0 ? -255 : rot == 1 ? __builtin_amdgcn_sbfe((int)rg, 3, 13) : rot == 2 ? (int)rg >> 19 : b >> 3;
    };
    const int v0 = nvalue(0);
    int nlo = v0, nhi = v0;
    bool same = true;
    for (int i = 1; i < 16; i++) {
        int v = nvalue(i);
        same &= v == v0;
        nlo = min(nlo, v);
        nhi = max(nhi, v);
    }
    PairFit best;
    best.sse = 0xFFFFFFFFu;
    best.idx = 0;
    best.c0 = best.c1 = 0;
    best.p0 = best.p1 = 0;
    if (same) {
        for (int k = 0; k < (1 << NB); k++) {
            const uint32_t ent = sv[((uint64_t)(cls * 4) * kSlots + slot_of(NB, k)) * 256 + (-v0)];
            const uint32_t er = ent >> 16;
            if (er * er < best.sse) {
                best.sse = er * er;
                best.idx = (uint64_t)k * 0x1111111111111111ull;
                best.c0 = ent & 255u;
                best.c1 = (ent >> 8) & 255u;
            }
        }
        best.sse *= 16u;
        return best;
    }
    int elo = -nhi, ehi = -nlo;   // least and greatest value
    for (int pass = 0; pass < 2; pass++) {
        const uint32_t e0 = S.q[cls * 2 * 256 + elo], e1 = S.q[cls * 2 * 256 + ehi];
        const int d0 = CODES ? (int)(e0 >> 8) : (int)(e0 >> 6), d1 = CODES ? (int)(e1 >> 8) : (int)(e1 >> 6);
        // entry k as 32 p (against the negated value) and 16 p^2 + k
        int pal[1 << NB], pk[1 << NB];
#pragma unroll
        for (int k = 0; k < (1 << NB); k++) {
            const int pv = interp64(d0, d1, bc7_weight(NB, k));
            pal[k] = 32 * pv;
            pk[k] = 16 * (int)__builtin_amdgcn_udot4((uint32_t)pv, (uint32_t)pv, 0u, false) + k;
        }
        uint32_t sse = 0;
        uint64_t idx = 0;
        int A = 0, B = 0, AB2 = 0, nSA = 0, nSB = 0;
        for (int i = 0; i < 16; i++) {
            const int x = nvalue(i);
            int kmin = 0x7FFFFFFF;
#pragma unroll
            for (int k = 0; k < (1 << NB); k++) kmin = min(kmin, mul_i24(x, pal[k]) + pk[k]);
            const uint32_t kb = (uint32_t)(kmin + 16 * x * x);   // 16 SSE + k
            sse += kb >> 4;
            idx |= (uint64_t)(kb & 15u) << (4 * i);
            const int w = bc7_weight(NB, (int)(kb & 15u)), a = 64 - w;
            A += a * a; B += w * w; AB2 += a * w; nSA += a * x; nSB += w * x;
        }
        if (sse < best.sse) {
            best.sse = sse;
            best.idx = idx;
            best.c0 = CODES ? e0 & 255u : 0u;
            best.c1 = CODES ? e1 & 255u : 0u;
        }
        if (pass == 1) break;
        const double det = (double)A * (double)B - (double)AB2 * (double)AB2;
        if (det == 0.0) break;
        // numerators of the positive values (the negated sums flip their sign)
        double n0 = -64.0 * ((double)B * (double)nSA - (double)AB2 * (double)nSB);
        double n1 = -64.0 * ((double)A * (double)nSB - (double)AB2 * (double)nSA);
        double q0 = floor(n0 / det + 0.5), q1 = floor(n1 / det + 0.5);
        elo = q0 < 0.0 ? 0 : (q0 > 255.0 ? 255 : (int)q0);
        ehi = q1 < 0.0 ? 0 : (q1 > 255.0 ? 255 : (int)q1);
    }
    return best;
}

// (e) the anchor texel's index must have its top bit clear; otherwise swap
// the endpoints (and p-bits) and mirror every member's index.
template <int NB>
__device__ __forceinline__ void anchor_fix(PairFit &f, uint32_t mask, int anchor)
{
    if (!((f.idx >> (4 * anchor + NB - 1)) & 1)) return;
    uint32_t t = f.c0; f.c0 = f.c1; f.c1 = t;
    int u = f.p0; f.p0 = f.p1; f.p1 = u;
    uint64_t spread = 0;
    for (uint32_t m = mask; m; m &= m - 1) spread |= (uint64_t)((1u << NB) - 1) << (4 * (__ffs(m) - 1));
    f.idx ^= spread;   // k -> (2^NB - 1) - k on the members
}

// ---- visiting order of the 3-subset partitions
//
// Of the 192 subset masks of the 64 three-subset partitions only 140 differ
// (36 of the 48 of partitions 0..15, the ones mode 0 also uses).  The search
// visits the partitions in the order below; a mask that recurs is fitted
// once and its SSE kept in an LDS slot of its lane until its last use.  This
// order (found offline by a local search) needs at most kSlots2 slots for
// mode 2 and kSlots0 for mode 0; a static check below recomputes both.
constexpr int kOrder3[64] = {62, 9,  2,  0,  60, 42, 61, 27, 38, 18, 46, 33, 51, 47, 55, 41,
                             31, 17, 63, 15, 23, 10, 36, 22, 8,  56, 29, 4,  3,  24, 6,  32,
                             25, 19, 14, 37, 34, 7,  26, 43, 52, 5,  54, 50, 20, 48, 1,  39,
                             58, 13, 35, 57, 53, 30, 21, 59, 49, 40, 28, 45, 16, 11, 44, 12};
constexpr int kSlots2 = 6, kSlots0 = 4;

__host__ __device__ constexpr uint32_t mask3_of(int p, int s)
{
    uint32_t m = 0;
    for (int i = 0; i < 16; i++) m |= (((kPart3[p] >> (2 * i)) & 3) == (uint32_t)s ? 1u : 0u) << i;
    return m;
}

// What the search does at visit t (partition kOrder3[t]), subset s, per mode:
//   kFit           fit the subset
//   kKeep | slot   fit it and keep the SSE in the slot (the mask recurs)
//   kTake | slot   take the SSE from the slot (fitted at an earlier visit)
constexpr uint8_t kFit = 0, kKeep = 0x40, kTake = 0x80;
struct Plan3 {
    uint8_t act[2][64][3];   // [0]: mode 2 (all partitions), [1]: mode 0 (partitions 0..15)
    int slots[2];            // slots each mode needs
};

constexpr Plan3 make_plan3()
{
    Plan3 P{};
    for (int mode = 0; mode < 2; mode++) {
        // each visit's mask, then its last visit
        uint32_t mk[192] = {};
        int pos[192] = {}, n = 0;
        for (int t = 0; t < 64; t++)
            for (int s = 0; s < 3; s++)
                if (mode == 0 || kOrder3[t] < 16) { mk[n] = mask3_of(kOrder3[t], s); pos[n] = t * 3 + s; n++; }
        bool used[8] = {};
        uint32_t held[8] = {};
        int most = 0;
        for (int q = 0; q < n; q++) {
            int later = -1, slot = -1;
            for (int r = q + 1; r < n; r++)
                if (mk[r] == mk[q]) { later = r; break; }
            for (int z = 0; z < 8; z++)
                if (used[z] && held[z] == mk[q]) slot = z;
            uint8_t a = kFit;
            if (slot >= 0) {
                a = (uint8_t)(kTake | slot);
                if (later < 0) used[slot] = false;   // last use
            } else if (later >= 0) {
                int z = 0;
                while (used[z]) z++;
                used[z] = true;
                held[z] = mk[q];
                a = (uint8_t)(kKeep | z);
                int live = 0;
                for (int y = 0; y < 8; y++) live += used[y] ? 1 : 0;
                most = live > most ? live : most;
            }
            P.act[mode][pos[q] / 3][pos[q] % 3] = a;
        }
        P.slots[mode] = most;
    }
    return P;
}
constexpr Plan3 kPlan3 = make_plan3();
static_assert(kPlan3.slots[0] <= kSlots2 && kPlan3.slots[1] <= kSlots0, "3-subset visiting order needs more slots");

// ---- pass 1: best key over one candidate group
//
// The principal axis and the extreme texels of a subset depend only on the
// partition, so they are found once and shared by every mode with that
// partition.  The candidates fall into three groups by partition shape; each
// group is its own kernel (smaller register footprint), and the block's key
// is the minimum over the groups.
__device__ __forceinline__ void consider(uint32_t sse, int ci, uint32_t &best)
{
    best = min(best, (sse << 9) | (uint32_t)ci);
}

// Per-lane SSE slots of the 3-subset search (kSlots2 for mode 2, then
// kSlots0 for mode 0), one column per lane.
typedef uint32_t Cache3[kSlots2 + kSlots0][kWG];

template <int GROUP>
__device__ __forceinline__ uint32_t search_group(const TexLds &S, Cache3 &cache, uint32_t mode_mask,
                                                 const uint32_t *sv)
{
    uint32_t best = 0xFFFFFFFFu;
    const Sums tot = GROUP == 0 ? subset_sums(S, 0xFFFFu, 0) : Sums{};
    if (GROUP == 0) {
        // 2-subset partitions: modes 1, 3, 7
        if (mode_mask & 0x8A)
            for (int p = 0; p < 64; p++) {
                const uint32_t m0 = mask2(p, 0), m1 = mask2(p, 1);
                const Sums s0 = subset_sums(S, m0, 0);
                const Prep P0 = prep_subset(S, m0, 0, s0), P1 = prep_subset(S, m1, 0, sums_minus(tot, s0));
                if (mode_mask & 0x02)
                    consider(fit_colour<6, 1, 3, true>(S, m0, 0, P0, sv).sse + fit_colour<6, 1, 3, true>(S, m1, 0, P1, sv).sse,
                             16 + p, best);
                if (mode_mask & 0x08)
                    consider(fit_colour<7, 2, 2, true>(S, m0, 0, P0, sv).sse + fit_colour<7, 2, 2, true>(S, m1, 0, P1, sv).sse,
                             144 + p, best);
                if (mode_mask & 0x80)
                    consider(fit_colour<5, 2, 2, true>(S, m0, 0, P0, sv).sse + fit_colour<5, 2, 2, true>(S, m1, 0, P1, sv).sse,
                             221 + p, best);
            }
    } else if (GROUP == 1) {
        // 3-subset partitions: mode 0 (partitions 0..15), mode 2; recurring
        // subset masks are fitted once (see kPlan3)
        const bool on2 = mode_mask & 0x04, on0 = mode_mask & 0x01;
        if (on0 || on2)
            for (int t = 0; t < 64; t++) {
                const int p = kOrder3[t];
                if (!on2 && p >= 16) continue;
                const bool with0 = on0 && p < 16;
                uint32_t e2 = 0, e0 = 0;
#pragma unroll 1
                for (int s = 0; s < 3; s++) {
                    const uint32_t msk = mask3(p, s);
                    const int a2 = kPlan3.act[0][t][s], a0 = kPlan3.act[1][t][s];
                    const bool fit2 = on2 && !(a2 & kTake), fit0 = with0 && !(a0 & kTake);
                    uint32_t v2 = 0, v0 = 0;
                    if (on2 && (a2 & kTake)) v2 = cache[a2 & 15][threadIdx.x];
                    if (with0 && (a0 & kTake)) v0 = cache[kSlots2 + (a0 & 15)][threadIdx.x];
                    if (fit2 || fit0) {
                        const Prep P = prep_subset(S, msk, 0);
                        if (fit2) {
                            v2 = fit_colour<5, 0, 2, true>(S, msk, 0, P, sv).sse;
                            if (a2 & kKeep) cache[a2 & 15][threadIdx.x] = v2;
                        }
                        if (fit0) {
                            v0 = fit_colour<4, 2, 3, true>(S, msk, 0, P, sv).sse;
                            if (a0 & kKeep) cache[kSlots2 + (a0 & 15)][threadIdx.x] = v0;
                        }
                    }
                    e2 += v2;
                    e0 += v0;
                }
                if (on2) consider(e2, 80 + p, best);
                if (with0) consider(e0, p, best);
            }
    } else {
        // one subset: mode 6, and modes 4 / 5 for every rotation
        if (mode_mask & 0x70)
            for (int r = 0; r < 4; r++) {
                if (r > 0 && !(mode_mask & 0x30)) break;
                const Prep P = prep_subset(S, 0xFFFFu, r);
                if (r == 0 && (mode_mask & 0x40)) consider(fit_colour<7, 2, 4, true>(S, 0xFFFFu, 0, P, sv).sse, 220, best);
                if (mode_mask & 0x10) {
                    uint32_t s0 = fit_colour<5, 0, 2, true>(S, 0xFFFFu, r, P, sv).sse;
                    uint32_t s1 = fit_colour<5, 0, 3, true>(S, 0xFFFFu, r, P, sv).sse;
                    if (r) { s0 += fit_scalar<6, 3, false>(S, r, sv).sse; s1 += fit_scalar<6, 2, false>(S, r, sv).sse; }
                    consider(s0, 208 + 2 * r, best);
                    consider(s1, 209 + 2 * r, best);
                }
                if (mode_mask & 0x20) {
                    uint32_t s5 = fit_colour<7, 0, 2, true>(S, 0xFFFFu, r, P, sv).sse;
                    if (r) s5 += fit_scalar<8, 2, false>(S, r, sv).sse;
                    consider(s5, 216 + r, best);
                }
            }
    }
    return best;
}

// ---- pass 2: re-fit the winner (same arithmetic) and lay out its bits
struct Writer {
    uint64_t lo = 0, hi = 0;
    int pos = 0;
    __device__ void put(uint32_t v, int n)
    {
        uint64_t x = (uint64_t)v & ((1ull << n) - 1);
        if (pos >= 64) hi |= x << (pos - 64);
        else {
            lo |= x << pos;
            if (pos + n > 64) hi |= x >> (64 - pos);
        }
        pos += n;
    }
};

template <int M, int CB, int PB, int NB>
__device__ void emit_partitioned(const TexLds &S, int p, const uint32_t *sv, Writer &w)
{
    constexpr Bc7Mode md = bc7_mode(M);
    constexpr int NS = md.ns;
    PairFit f[NS];
    uint32_t msk[NS];
    int anc[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        msk[s] = NS == 3 ? mask3(p, s) : mask2(p, s);
        anc[s] = bc7_anchor(NS, p, s);
        const Prep P = prep_subset(S, msk[s], 0);
        f[s] = fit_colour<CB, PB, NB>(S, msk[s], 0, P, sv);
        anchor_fix<NB>(f[s], msk[s], anc[s]);
    }
    w.put(1u << M, M + 1);
    w.put((uint32_t)p, md.partbits);
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put(f[s].c0 >> (8 * c), CB); w.put(f[s].c1 >> (8 * c), CB); }
    if (md.ab)   // alpha is not coded for these colour blocks: all-ones fields
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put((1u << md.ab) - 1, md.ab); w.put((1u << md.ab) - 1, md.ab); }
    if (PB == 2)
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put(f[s].p0, 1); w.put(f[s].p1, 1); }
    else if (PB == 1)
#pragma unroll
        for (int s = 0; s < NS; s++) w.put(f[s].p0, 1);
    // members' indices live in their own subset's fit: merge them
    uint64_t idx = 0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        uint64_t sel = 0;
        for (uint32_t m = msk[s]; m; m &= m - 1) sel |= (uint64_t)15 << (4 * (__ffs(m) - 1));
        idx |= f[s].idx & sel;
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
        bool anchored = false;
#pragma unroll
        for (int q = 0; q < NS; q++) anchored |= anc[q] == i;
        w.put((uint32_t)((idx >> (4 * i)) & 15), NB - (anchored ? 1 : 0));
    }
}

// Modes 4 and 5: one colour pair plus a scalar pair, rotation r.
template <int M, int CB, int AB, int CNB, int SNB>
__device__ void emit_rotated(const TexLds &S, int r, int sel, const uint32_t *sv, Writer &w)
{
    const Prep P = prep_subset(S, 0xFFFFu, r);
    PairFit fc = fit_colour<CB, 0, CNB>(S, 0xFFFFu, r, P, sv);
    anchor_fix<CNB>(fc, 0xFFFFu, 0);
    PairFit fs = fit_scalar<AB, SNB, true>(S, r, sv);
    anchor_fix<SNB>(fs, 0xFFFFu, 0);
    w.put(1u << M, M + 1);
    w.put((uint32_t)r, 2);
    if (M == 4) w.put((uint32_t)sel, 1);
#pragma unroll
    for (int c = 0; c < 3; c++) { w.put(fc.c0 >> (8 * c), CB); w.put(fc.c1 >> (8 * c), CB); }
    w.put(fs.c0, AB);
    w.put(fs.c1, AB);
    // primary index set (2 bits) first, then the secondary set; index
    // selection 1 stores the scalar indices in the primary set
    const uint64_t first = (M == 4 && sel) ? fs.idx : fc.idx;
    const uint64_t second = (M == 4 && sel) ? fc.idx : fs.idx;
    constexpr int NB1 = 2, NB2 = (M == 4) ? 3 : 2;
#pragma unroll
    for (int i = 0; i < 16; i++) w.put((uint32_t)((first >> (4 * i)) & 15), NB1 - (i == 0));
#pragma unroll
    for (int i = 0; i < 16; i++) w.put((uint32_t)((second >> (4 * i)) & 15), NB2 - (i == 0));
}

// Bits of a winning candidate of mode M.
template <int M>
__device__ __forceinline__ void emit(const TexLds &S, int ci, const uint32_t *sv, uint64_t &lo, uint64_t &hi)
{
    int m, p, r, s;
    candidate(ci, m, p, r, s);
    Writer w;
    if (M == 0) emit_partitioned<0, 4, 2, 3>(S, p, sv, w);
    else if (M == 1) emit_partitioned<1, 6, 1, 3>(S, p, sv, w);
    else if (M == 2) emit_partitioned<2, 5, 0, 2>(S, p, sv, w);
    else if (M == 3) emit_partitioned<3, 7, 2, 2>(S, p, sv, w);
    else if (M == 4) {
        if (s == 0) emit_rotated<4, 5, 6, 2, 3>(S, r, 0, sv, w);
        else emit_rotated<4, 5, 6, 3, 2>(S, r, 1, sv, w);
    } else if (M == 5) emit_rotated<5, 7, 8, 2, 2>(S, r, 0, sv, w);
    else if (M == 6) {
        const Prep P = prep_subset(S, 0xFFFFu, 0);
        PairFit f = fit_colour<7, 2, 4>(S, 0xFFFFu, 0, P, sv);
        anchor_fix<4>(f, 0xFFFFu, 0);
        w.put(1u << 6, 7);
#pragma unroll
        for (int c = 0; c < 3; c++) { w.put(f.c0 >> (8 * c), 7); w.put(f.c1 >> (8 * c), 7); }
        w.put(127, 7); w.put(127, 7);   // alpha not coded: all-ones fields
        w.put(f.p0, 1); w.put(f.p1, 1);
#pragma unroll
        for (int i = 0; i < 16; i++) w.put((uint32_t)((f.idx >> (4 * i)) & 15), 4 - (i == 0));
    } else emit_partitioned<7, 5, 2, 2>(S, p, sv, w);
    lo = w.lo;
    hi = w.hi;
}

struct Bc7Launch {
    EncodeArgs a;
    Tables T;
    WorkSplit w;
};

// The nearest-code table into LDS: 64-scaled values for the search,
// code | value << 8 for the emit pass.
__device__ __forceinline__ void stage_table(TexLds &S, const uint16_t *table)
{
    for (int q = threadIdx.x; q < kQEntries / 2; q += kWG)
        reinterpret_cast<uint32_t *>(S.q)[q] = reinterpret_cast<const uint32_t *>(table)[q];
}

// This lane's block (zeros when not live) into its LDS column in the -8
// scaled layout.  The caller brackets it with barriers.
__device__ __forceinline__ void stage_texels(TexLds &S, const uint8_t *src, bool live)
{
    uint32_t t[16];
#pragma unroll
    for (int i = 0; i < 16; i++) t[i] = 0;
    if (live) {
        const uint4 *p = reinterpret_cast<const uint4 *>(src);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            uint4 v = p[q];
            t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int r = (int)(t[i] & 255u), g = (int)((t[i] >> 8) & 255u), bb = (int)((t[i] >> 16) & 255u);
        S.rg[i][threadIdx.x] = ((uint32_t)(kScaleNeg * r) & 0xFFFFu) | ((uint32_t)(kScaleNeg * g) << 16);
        S.bx[i][threadIdx.x] = kScaleNeg * bb;
    }
}

// Items of the work split handled by this workgroup: one (its own index)
// without a queue, else popped from the queue until exhausted.  Every
// workgroup leaves the loop once the counter passes the last item.
struct ItemLoop {
    uint32_t item, n_items;
    __device__ __forceinline__ ItemLoop(const WorkSplit &w, uint64_t total, uint32_t round, uint32_t *s_item)
    {
        n_items = (uint32_t)((total + (uint64_t)w.item_rounds * round - 1) / ((uint64_t)w.item_rounds * round));
        item = blockIdx.x;
        if (w.queue) {
            if (threadIdx.x == 0) *s_item = atomicAdd(w.queue, 1u);
            __syncthreads();
            item = *s_item;
        }
    }
    __device__ __forceinline__ bool next(const WorkSplit &w, uint32_t *s_item)
    {
        if (!w.queue) return false;
        __syncthreads();   // every thread has read *s_item
        if (threadIdx.x == 0) *s_item = atomicAdd(w.queue, 1u);
        __syncthreads();
        item = *s_item;
        return item < n_items;
    }
};

// Pass 1: the best key of every block over the candidate groups in GMASK
// (bit 0: 2-subset modes, bit 1: 3-subset modes, bit 2: 1-subset modes),
// min-combined into the block's key word (set to all-ones beforehand) with
// an atomic minimum, so kernels and work items may run in any order.
// GMASK == 8 makes each (group, rounds) pair a work item of its own, heavy
// groups first, so one launch covers all groups and ends on light items.
template <int GMASK>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(3))) void k_bc7_search(Bc7Launch L)
{
    __shared__ TexLds S;
    __shared__ Cache3 cache;
    __shared__ uint32_t s_item;
    constexpr bool kItems = GMASK == 8;
    const EncodeArgs &a = L.a;
    const uint64_t rounds = a.total / kWG;
    const uint64_t per_group = (rounds + L.w.item_rounds - 1) / L.w.item_rounds;   // items per group
    stage_table(S, L.T.near64);
    ItemLoop it(L.w, kItems ? 3 * per_group * L.w.item_rounds * kWG : a.total, kWG, &s_item);
    if (it.item >= it.n_items) return;
    do {
        const uint32_t group = kItems ? (uint32_t)(it.item / per_group) : 0u;
        const uint64_t first = kItems ? (it.item % per_group) * L.w.item_rounds : (uint64_t)it.item * L.w.item_rounds;
        for (uint32_t r = 0; r < L.w.item_rounds; r++) {
            const uint64_t g0 = (first + r) * kWG;
            if (g0 >= a.total) break;
            const BlockRun run = a.run[find_run(a.run, a.nrun, g0)];
            const uint64_t b = g0 - run.gbase + threadIdx.x;
            const bool live = b < run.nblk;
            __syncthreads();   // the previous round's LDS reads are done
            stage_texels(S, run.src + b * 64, live);
            __syncthreads();
            if (__ballot(live) == 0) continue;
            if (live) {
                uint32_t key = ~0u;
                if (kItems) {
                    key = group == 0 ? search_group<0>(S, cache, a.mode_mask, L.T.sv)
                                     : group == 1 ? search_group<1>(S, cache, a.mode_mask, L.T.sv)
                                                  : search_group<2>(S, cache, a.mode_mask, L.T.sv);
                } else {
                    if (GMASK & 1) key = min(key, search_group<0>(S, cache, a.mode_mask, L.T.sv));
                    if (GMASK & 2) key = min(key, search_group<1>(S, cache, a.mode_mask, L.T.sv));
                    if (GMASK & 4) key = min(key, search_group<2>(S, cache, a.mode_mask, L.T.sv));
                }
                atomicMin(a.keys + g0 + threadIdx.x, key);
            }
        }
    } while (it.next(L.w, &s_item));
}

// Between the passes: bucket the blocks by the mode of their winner, so that
// the emit kernel of each mode runs full waves of that mode.  Order inside a
// bucket does not matter: every block is emitted independently.  Padding
// indices (key all-ones) join no bucket.
__device__ __forceinline__ int mode_of_candidate(int ci)
{
    return ci < 16 ? 0 : ci < 80 ? 1 : ci < 144 ? 2 : ci < 208 ? 3 : ci < 216 ? 4 : ci < 220 ? 5 : ci < 221 ? 6 : 7;
}

// Per-workgroup mode counts (LDS atomics), written to wgcount[wg][8]; each
// block's final SSE (key >> 9) is added into its run's sum here.  Runs
// start at multiples of 256 blocks, so a workgroup lies in one run: its
// SSEs are summed in LDS first and reach the run's sum as one atomic (per
// wave, a thousand waves of one band would queue on the same address).
__global__ __launch_bounds__(kWG) void k_bc7_bucket_count(EncodeArgs a, uint32_t *wgcount)
{
    __shared__ uint32_t c[8];
    __shared__ unsigned long long s_sse;
    if (threadIdx.x < 8) c[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_sse = 0;
    __syncthreads();
    const uint64_t g0 = (uint64_t)blockIdx.x * kWG, g = g0 + threadIdx.x;
    const uint32_t key = g < a.total ? a.keys[g] : ~0u;
    const bool live = key != ~0u;
    if (live) atomicAdd(&c[mode_of_candidate((int)(key & 511u))], 1u);
    const BlockRun run = a.run[find_run(a.run, a.nrun, g0)];
    if (run.sse) {
        unsigned long long x = live ? (unsigned long long)(key >> 9) : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if ((threadIdx.x & 63) == 0) atomicAdd(&s_sse, x);
    }
    __syncthreads();
    if (threadIdx.x < 8) wgcount[(uint64_t)blockIdx.x * 8 + threadIdx.x] = c[threadIdx.x];
    if (threadIdx.x == 0 && run.sse && s_sse) atomicAdd(&run.sse[0], s_sse);
}

// Exclusive scan of wgcount down each mode's column, then the buckets:
// count[m] = bucket size, count[8 + m] = its first list slot.  One
// workgroup: each thread sums a run of rows, the run totals are scanned in
// LDS, and each thread rewrites its rows.
__global__ __launch_bounds__(256) void k_bc7_bucket_scan(uint32_t *wgcount, uint32_t nwg, uint32_t *count)
{
    __shared__ uint32_t part[256][8];
    __shared__ uint32_t tot[8];
    const uint32_t t = threadIdx.x, per = (nwg + 255) / 256;
    const uint32_t r0 = min(nwg, t * per), r1 = min(nwg, r0 + per);
    uint32_t acc[8];
#pragma unroll
    for (int m = 0; m < 8; m++) acc[m] = 0;
    for (uint32_t r = r0; r < r1; r++)
#pragma unroll
        for (int m = 0; m < 8; m++) acc[m] += wgcount[(uint64_t)r * 8 + m];
#pragma unroll
    for (int m = 0; m < 8; m++) part[t][m] = acc[m];
    __syncthreads();
    if (t < 8) {
        uint32_t run = 0;
        for (int u = 0; u < 256; u++) {
            uint32_t v = part[u][t];
            part[u][t] = run;
            run += v;
        }
        tot[t] = run;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; m++) {
        uint32_t run = part[t][m];
        for (uint32_t r = r0; r < r1; r++) {
            uint32_t v = wgcount[(uint64_t)r * 8 + m];
            wgcount[(uint64_t)r * 8 + m] = run;
            run += v;
        }
    }
    if (t < 8) {
        uint32_t start = 0;
        for (uint32_t q = 0; q < t; q++) start += tot[q];
        count[t] = tot[t];
        count[8 + t] = start;
    }
}

__global__ __launch_bounds__(kWG) void k_bc7_bucket_fill(const uint32_t *keys, uint64_t total, const uint32_t *wgoff,
                                                         const uint32_t *count, uint32_t *list)
{
    __shared__ uint32_t c[8];
    if (threadIdx.x < 8) c[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t g = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (g >= total || keys[g] == ~0u) return;
    const int m = mode_of_candidate((int)(keys[g] & 511u));
    const uint32_t rank = atomicAdd(&c[m], 1u);
    list[count[8 + m] + wgoff[(uint64_t)blockIdx.x * 8 + m] + rank] = (uint32_t)g;
}

// Pass 2: re-fit each block's winning candidate and write its bits; one
// kernel per mode over that mode's bucket (small code, full waves).
template <int M>
__global__ __launch_bounds__(kWG) void k_bc7_emit(Bc7Launch L)
{
    __shared__ TexLds S;
    const EncodeArgs &a = L.a;
    const uint32_t *list = a.keys + a.total, *count = a.keys + 2 * a.total;
    const uint32_t n = count[M], off = count[8 + M];
    const uint64_t e = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if ((uint64_t)blockIdx.x * kWG >= n) return;   // whole workgroup past the bucket
    const bool live = e < n;
    const uint64_t g = live ? list[off + e] : a.run[0].gbase;
    const BlockRun run = a.run[find_run(a.run, a.nrun, g)];
    const uint64_t b = g - run.gbase;
    stage_table(S, L.T.nearest);
    stage_texels(S, run.src + b * 64, live);   // lanes past the bucket stage zeros
    __syncthreads();
    if (!live) return;
    const uint32_t key = a.keys[g];
    uint64_t lo, hi;
    emit<M>(S, (int)(key & 511u), L.T.sv, lo, hi);
    *reinterpret_cast<ulonglong2 *>(run.dst + b * 16) = make_ulonglong2(lo, hi);
}

// ---- host-side table construction
struct HostTables {
    std::vector<uint16_t> nearest;  // [10][2][256]
    std::vector<uint16_t> near64;   // [10][2][256]
    std::vector<uint32_t> sv;       // [10][4][kSlots][256]
};

void build_nearest(HostTables &H)
{
    H.nearest.assign(10 * 2 * 256, 0);
    for (int cb = 4; cb <= 8; cb++)
        for (int pb = 0; pb < 2; pb++)
            for (int p = 0; p < 2; p++) {
                if (!pb && p) continue;
                const int nc = 1 << cb;
                uint16_t *row = &H.nearest[(cls_of(cb, pb) * 2 + p) * 256];
                for (int t = 0; t < 256; t++) {
                    int bc = 0, bd = 1 << 30;
                    for (int c = 0; c < nc; c++) {
                        int d = ep_value(c, p, cb, pb) - t;
                        d = d < 0 ? -d : d;
                        if (d < bd) { bd = d; bc = c; }
                    }
                    row[t] = (uint16_t)(bc | (ep_value(bc, p, cb, pb) << 8));
                }
            }
    H.near64.resize(H.nearest.size());
    for (size_t q = 0; q < H.nearest.size(); q++) H.near64[q] = (uint16_t)((H.nearest[q] >> 8) << 6);
}

// Best pair per target value v for one (class, p-bits, weight): first the
// best pair (by |c0-c1|, c0, c1) reaching each interpolated value u, then for
// each v the nearest reachable u (both sides of v compared by the same key).
void build_sv_entry(uint32_t *row, int cb, int pb, int p0, int p1, int wgt)
{
    const int nc = 1 << cb;
    int bestpair[256];
    for (int u = 0; u < 256; u++) bestpair[u] = -1;
    auto better = [&](int a0, int a1, int b0, int b1) {   // is (a0,a1) ahead of (b0,b1)?
        int da = a0 > a1 ? a0 - a1 : a1 - a0, db = b0 > b1 ? b0 - b1 : b1 - b0;
        if (da != db) return da < db;
        if (a0 != b0) return a0 < b0;
        return a1 < b1;
    };
    for (int a = 0; a < nc; a++)
        for (int b = 0; b < nc; b++) {
            int u = interp64(ep_value(a, p0, cb, pb), ep_value(b, p1, cb, pb), wgt);
            int cur = bestpair[u];
            if (cur < 0 || better(a, b, cur >> 8, cur & 255)) bestpair[u] = (a << 8) | b;
        }
    for (int v = 0; v < 256; v++) {
        for (int d = 0; d < 256; d++) {
            int pick = -1;
            for (int side = 0; side < 2; side++) {
                int u = side ? v + d : v - d;
                if (u < 0 || u > 255 || bestpair[u] < 0) continue;
                int pr = bestpair[u];
                if (pick < 0 || better(pr >> 8, pr & 255, pick >> 8, pick & 255)) pick = pr;
            }
            if (pick >= 0) {
                row[v] = (uint32_t)(pick >> 8) | ((uint32_t)(pick & 255) << 8) | ((uint32_t)d << 16);
                break;
            }
        }
    }
}

void build_sv(HostTables &H)
{
    H.sv.assign((size_t)10 * 4 * kSlots * 256, 0);
    struct Use { int cb, pb, nb; };
    const Use uses[] = {{4, 2, 3}, {6, 1, 3}, {5, 0, 2}, {7, 2, 2}, {5, 0, 3}, {6, 0, 3}, {6, 0, 2},
                        {7, 0, 2}, {8, 0, 2}, {7, 2, 4}, {5, 2, 2}};
    for (const Use &u : uses) {
        const int npc = u.pb == 2 ? 4 : u.pb == 1 ? 2 : 1;
        for (int pc = 0; pc < npc; pc++) {
            int p0 = u.pb == 2 ? (pc & 1) : u.pb == 1 ? pc : 0;
            int p1 = u.pb == 2 ? (pc >> 1) : u.pb == 1 ? pc : 0;
            for (int k = 0; k < (1 << u.nb); k++) {
                uint32_t *row = &H.sv[(((size_t)cls_of(u.cb, u.pb) * 4 + p0 + 2 * p1) * kSlots + slot_of(u.nb, k)) * 256];
                build_sv_entry(row, u.cb, u.pb, p0, p1, bc7_weight(u.nb, k));
            }
        }
    }
}

}  // namespace

// Device copies of the tables, one set per device, made once per device
// (under a lock: contexts may be created from several threads).
static void *g_tab[kMaxDevices];
static std::mutex g_tab_lock;

hipError_t upload_bc7_tables(int device, hipStream_t st)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_tab_lock);
    if (g_tab[device]) return hipSuccess;
    static HostTables H;
    if (H.nearest.empty()) { build_nearest(H); build_sv(H); }
    size_t nb = H.nearest.size() * 2, sb = H.sv.size() * 4;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, 2 * nb + sb);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(p, H.nearest.data(), nb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync((char *)p + nb, H.near64.data(), nb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync((char *)p + 2 * nb, H.sv.data(), sb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { (void)hipFree(p); return e; }
    g_tab[device] = p;
    return hipSuccess;
}

hipError_t launch_bc7_encode(const EncodeArgs &a, const WorkSplit *w3, uint32_t split, hipStream_t st,
                             hipEvent_t searched)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (!g_tab[dev]) return hipErrorNotInitialized;
    if (a.total == 0) return hipSuccess;
    if (split > 3) return hipErrorInvalidValue;
    Bc7Launch L;
    L.a = a;
    L.T.nearest = static_cast<const uint16_t *>(g_tab[dev]);
    L.T.near64 = L.T.nearest + kQEntries;
    L.T.sv = reinterpret_cast<const uint32_t *>(L.T.near64 + kQEntries);
    const uint32_t nwg = (uint32_t)(a.total / kWG);
    const dim3 sgrid(nwg);
    // every key word starts all-ones (padding indices keep it)
    if ((e = launch_fill_u64(reinterpret_cast<unsigned long long *>(a.keys), a.total / 2, ~0ull, st)) != hipSuccess)
        return e;
    auto launch = [&](int q, auto kernel, const char *name) -> hipError_t {
        L.w = w3[q];
        const uint32_t per = (uint32_t)((nwg + L.w.item_rounds - 1) / L.w.item_rounds);
        dim3 grid(L.w.queue ? L.w.grid : (split == 3 ? 3 * per : per));
        if (L.w.queue) {
            hipError_t f = launch_fill_u64(reinterpret_cast<unsigned long long *>(L.w.queue), 1, 0, st);
            if (f != hipSuccess) return f;
        }
        GSBC_LAUNCH(name, kernel, grid, dim3(kWG), 0, st, L);
        return hipGetLastError();
    };
    if (split == 0) {
        if ((e = launch(0, k_bc7_search<1>, "bc7_search_2subset")) != hipSuccess) return e;
        if ((e = launch(1, k_bc7_search<2>, "bc7_search_3subset")) != hipSuccess) return e;
        if ((e = launch(2, k_bc7_search<4>, "bc7_search_1subset")) != hipSuccess) return e;
    } else if (split == 1) {
        if ((e = launch(0, k_bc7_search<1>, "bc7_search_2subset")) != hipSuccess) return e;
        if ((e = launch(1, k_bc7_search<6>, "bc7_search_3subset_1subset")) != hipSuccess) return e;
    } else if (split == 2) {
        if ((e = launch(0, k_bc7_search<7>, "bc7_search_all")) != hipSuccess) return e;
    } else {
        if ((e = launch(0, k_bc7_search<8>, "bc7_search_items")) != hipSuccess) return e;
    }
    if (searched && (e = hipEventRecord(searched, st)) != hipSuccess) return e;
    // key scratch: keys[total] | list[total] | count[8] start[8] | wgcount[nwg][8]
    uint32_t *count = a.keys + 2 * a.total, *wgcount = count + 16;
    GSBC_LAUNCH("bc7_bucket", k_bc7_bucket_count, sgrid, dim3(kWG), 0, st, a, wgcount);
    GSBC_LAUNCH("bc7_bucket", k_bc7_bucket_scan, dim3(1), dim3(256), 0, st, wgcount, nwg, count);
    GSBC_LAUNCH("bc7_bucket", k_bc7_bucket_fill, sgrid, dim3(kWG), 0, st, a.keys, a.total, wgcount, count,
                a.keys + a.total);
    L.w = w3[0];
    if (a.mode_mask & 0x01) GSBC_LAUNCH("bc7_emit_m0", k_bc7_emit<0>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x02) GSBC_LAUNCH("bc7_emit_m1", k_bc7_emit<1>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x04) GSBC_LAUNCH("bc7_emit_m2", k_bc7_emit<2>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x08) GSBC_LAUNCH("bc7_emit_m3", k_bc7_emit<3>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x10) GSBC_LAUNCH("bc7_emit_m4", k_bc7_emit<4>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x20) GSBC_LAUNCH("bc7_emit_m5", k_bc7_emit<5>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x40) GSBC_LAUNCH("bc7_emit_m6", k_bc7_emit<6>, sgrid, dim3(kWG), 0, st, L);
    if (a.mode_mask & 0x80) GSBC_LAUNCH("bc7_emit_m7", k_bc7_emit<7>, sgrid, dim3(kWG), 0, st, L);
    return hipGetLastError();
}

}  // namespace gsbc
