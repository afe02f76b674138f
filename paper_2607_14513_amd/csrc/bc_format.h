// bc_format.h -- BC1 / BC7 format constants and texel decoders for the
// gfx950 kernels (D3D11 BC1 and BC7 block formats, the fixed-rate BTC
// schemes of Sec. III-A/B of Said & Rauwendaal).
//
// The BC7 partition maps and anchor texels are transcribed from the public
// BC7/BPTC format specification.  2-subset maps are 16-bit masks (bit i =
// subset of texel i); 3-subset maps are packed at compile time from their
// row strings into 2 bits per texel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsbc {

// ------------------------------------------------------------------ BC7 modes
struct Bc7Mode {
    int ns;        // subsets
    int partbits;  // partition field width
    int rotbits;   // rotation field width
    int selbits;   // index-selection field width
    int cb;        // colour endpoint bits per channel
    int ab;        // alpha endpoint bits (0: none)
    int pb;        // p-bits: 0 none, 1 one per subset, 2 one per endpoint
    int ib;        // primary index bits
    int ib2;       // secondary index bits (0: none)
};

__host__ __device__ constexpr Bc7Mode bc7_mode(int m)
{
    return m == 0 ? Bc7Mode{3, 4, 0, 0, 4, 0, 2, 3, 0}
         : m == 1 ? Bc7Mode{2, 6, 0, 0, 6, 0, 1, 3, 0}
         : m == 2 ? Bc7Mode{3, 6, 0, 0, 5, 0, 0, 2, 0}
         : m == 3 ? Bc7Mode{2, 6, 0, 0, 7, 0, 2, 2, 0}
         : m == 4 ? Bc7Mode{1, 0, 2, 1, 5, 6, 0, 2, 3}
         : m == 5 ? Bc7Mode{1, 0, 2, 0, 7, 8, 0, 2, 2}
         : m == 6 ? Bc7Mode{1, 0, 0, 0, 7, 7, 2, 4, 0}
                  : Bc7Mode{2, 6, 0, 0, 5, 5, 2, 2, 0};
}

// Interpolation weight of index i with n index bits: round(64 i / (2^n - 1)).
__host__ __device__ constexpr int bc7_weight(int n, int i)
{
    return (128 * i + ((1 << n) - 1)) / (2 * ((1 << n) - 1));
}

// The same weights for n and i known only at run time (the decoders): the
// table bytes, little end first, taken by one 64-bit shift instead of a
// division by 2 (2^n - 1).
__host__ __device__ constexpr int bc7_weight_packed(int n, int i)
{
    const uint64_t lo = n == 2 ? 0x402B1500ull : n == 3 ? 0x40372E251B120900ull : 0x1E1A15110D090400ull;
    const uint64_t hi = 0x403C37332F2B2622ull;   // n = 4, indices 8..15
    return (int)(((i < 8 ? lo : hi) >> (8 * (i & 7))) & 255u);
}

__host__ __device__ constexpr bool bc7_weights_packed_ok()
{
    for (int n = 2; n <= 4; n++)
        for (int i = 0; i < (1 << n); i++)
            if (bc7_weight_packed(n, i) != bc7_weight(n, i)) return false;
    return true;
}
static_assert(bc7_weights_packed_ok(), "packed BC7 weight tables");

__host__ __device__ constexpr int interp64(int e0, int e1, int w)
{
    return ((64 - w) * e0 + w * e1 + 32) >> 6;
}

// Expand an n-bit value (5 <= n <= 8) to 8 bits by replicating its top bits.
__host__ __device__ constexpr int expand_bits(int v, int n)
{
    return n >= 8 ? v : (v << (8 - n)) | (v >> (2 * n - 8));
}

// ------------------------------------------------------------ partition maps
static __constant__ uint16_t kPart2[64] = {
    0xCCCC, 0x8888, 0xEEEE, 0xECC8, 0xC880, 0xFEEC, 0xFEC8, 0xEC80,
    0xC800, 0xFFEC, 0xFE80, 0xE800, 0xFFE8, 0xFF00, 0xFFF0, 0xF000,
    0xF710, 0x008E, 0x7100, 0x08CE, 0x008C, 0x7310, 0x3100, 0x8CCE,
    0x088C, 0x3110, 0x6666, 0x366C, 0x17E8, 0x0FF0, 0x718E, 0x399C,
    0xAAAA, 0xF0F0, 0x5A5A, 0x33CC, 0x3C3C, 0x55AA, 0x9696, 0xA55A,
    0x73CE, 0x13C8, 0x324C, 0x3BDC, 0x6996, 0xC33C, 0x9966, 0x0660,
    0x0272, 0x04E4, 0x4E40, 0x2720, 0xC936, 0x936C, 0x39C6, 0x639C,
    0x9336, 0x9CC6, 0x817E, 0xE718, 0xCCF0, 0x0FCC, 0x7744, 0xEE22,
};

__host__ __device__ constexpr uint32_t pack_row3(const char *r)
{
    uint32_t v = 0;
    for (int i = 0; i < 16; i++) v |= (uint32_t)(r[i] - '0') << (2 * i);
    return v;
}

// (constexpr: the encoder plans its visiting order from it at compile time)
constexpr uint32_t kPart3[64] = {
    pack_row3("0011001102212222"), pack_row3("0001001122112221"), pack_row3("0000200122112211"),
    pack_row3("0222002200110111"), pack_row3("0000000011221122"), pack_row3("0011001100220022"),
    pack_row3("0022002211111111"), pack_row3("0011001122112211"), pack_row3("0000000011112222"),
    pack_row3("0000111111112222"), pack_row3("0000111122222222"), pack_row3("0012001200120012"),
    pack_row3("0112011201120112"), pack_row3("0122012201220122"), pack_row3("0011011211221222"),
    pack_row3("0011200122002220"), pack_row3("0001001101121122"), pack_row3("0111001120012200"),
    pack_row3("0000112211221122"), pack_row3("0022002200221111"), pack_row3("0111011102220222"),
    pack_row3("0001000122212221"), pack_row3("0000001101220122"), pack_row3("0000110022102210"),
    pack_row3("0122012200110000"), pack_row3("0012001211222222"), pack_row3("0110122112210110"),
    pack_row3("0000011012211221"), pack_row3("0022110211020022"), pack_row3("0110011020022222"),
    pack_row3("0011012201220011"), pack_row3("0000200022112221"), pack_row3("0000000211221222"),
    pack_row3("0222002200120011"), pack_row3("0011001200220222"), pack_row3("0120012001200120"),
    pack_row3("0000111122220000"), pack_row3("0120120120120120"), pack_row3("0120201212010120"),
    pack_row3("0011220011220011"), pack_row3("0011112222000011"), pack_row3("0101010122222222"),
    pack_row3("0000000021212121"), pack_row3("0022112200221122"), pack_row3("0022001100220011"),
    pack_row3("0220122102201221"), pack_row3("0101222222220101"), pack_row3("0000212121212121"),
    pack_row3("0101010101012222"), pack_row3("0222011102220111"), pack_row3("0002111200021112"),
    pack_row3("0000211221122112"), pack_row3("0222011101110222"), pack_row3("0002111211120002"),
    pack_row3("0110011001102222"), pack_row3("0000000021122112"), pack_row3("0110011022222222"),
    pack_row3("0022001100110022"), pack_row3("0022112211220022"), pack_row3("0000000000002112"),
    pack_row3("0002000100020001"), pack_row3("0222122202221222"), pack_row3("0101222222222222"),
    pack_row3("0111201122012220"),
};

// Anchor texel of the second subset (2-subset partitions), and of the second
// and third subsets (3-subset partitions).  Subset 0's anchor is texel 0.
static __constant__ uint8_t kAnchor2[64] = {
    15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
    15, 2, 8, 2, 2, 8, 8, 15, 2, 8, 2, 2, 8, 8, 2, 2,
    15, 15, 6, 8, 2, 8, 15, 15, 2, 8, 2, 2, 2, 15, 15, 6,
    6, 2, 6, 8, 15, 15, 2, 2, 15, 15, 15, 15, 15, 2, 2, 15,
};
static __constant__ uint8_t kAnchor3b[64] = {
    3, 3, 15, 15, 8, 3, 15, 15, 8, 8, 6, 6, 6, 5, 3, 3,
    3, 3, 8, 15, 3, 3, 6, 10, 5, 8, 8, 6, 8, 5, 15, 15,
    8, 15, 3, 5, 6, 10, 8, 15, 15, 3, 15, 5, 15, 15, 15, 15,
    3, 15, 5, 5, 5, 8, 5, 10, 5, 10, 8, 13, 15, 12, 3, 3,
};
static __constant__ uint8_t kAnchor3c[64] = {
    15, 8, 8, 3, 15, 15, 3, 8, 15, 15, 15, 15, 15, 15, 15, 8,
    15, 8, 15, 3, 15, 8, 15, 8, 3, 15, 6, 10, 15, 15, 10, 8,
    15, 3, 15, 10, 10, 8, 9, 10, 6, 15, 8, 15, 3, 6, 6, 8,
    15, 3, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 3, 15, 15, 8,
};

// Partition-map and anchor access for the texel decoder.  The default reads
// the constant-memory tables above; a kernel can hand it a copy of them in
// LDS (Bc7PackedLut) so that its per-lane lookups wait on LDS instead of on
// the vector-memory counter its loads and stores share.
struct Bc7ConstLut {
    __device__ uint32_t part2(int p) const { return kPart2[p]; }
    __device__ uint32_t part3(int p) const { return kPart3[p]; }
    __device__ int anchor2(int p) const { return kAnchor2[p]; }
    __device__ int anchor3b(int p) const { return kAnchor3b[p]; }
    __device__ int anchor3c(int p) const { return kAnchor3c[p]; }
};

// The same tables as 128 words: word p (p < 64) = 2-subset mask | 2-subset
// anchor << 16 | 3-subset anchors << 20 and << 24; word 64 + p = 3-subset map.
constexpr int kBc7LutWords = 128;
__device__ inline uint32_t bc7_lut_word(int e)
{
    if (e >= 64) return kPart3[e - 64];
    return (uint32_t)kPart2[e] | (uint32_t)kAnchor2[e] << 16 | (uint32_t)kAnchor3b[e] << 20 |
           (uint32_t)kAnchor3c[e] << 24;
}

struct Bc7PackedLut {
    const uint32_t *w;   // kBc7LutWords words of bc7_lut_word
    __device__ uint32_t part2(int p) const { return w[p] & 0xFFFFu; }
    __device__ uint32_t part3(int p) const { return w[64 + p]; }
    __device__ int anchor2(int p) const { return (int)(w[p] >> 16) & 15; }
    __device__ int anchor3b(int p) const { return (int)(w[p] >> 20) & 15; }
    __device__ int anchor3c(int p) const { return (int)(w[p] >> 24) & 15; }
};

// Subset of texel i in partition p of an ns-subset mode.
template <class Lut>
__device__ inline int bc7_subset(int ns, int p, int i, const Lut &lut)
{
    if (ns == 1) return 0;
    if (ns == 2) return (lut.part2(p) >> i) & 1;
    return (lut.part3(p) >> (2 * i)) & 3;
}
__device__ inline int bc7_subset(int ns, int p, int i) { return bc7_subset(ns, p, i, Bc7ConstLut{}); }

// Anchor texel of subset s.
template <class Lut>
__device__ inline int bc7_anchor(int ns, int p, int s, const Lut &lut)
{
    if (s == 0) return 0;
    if (ns == 2) return lut.anchor2(p);
    return s == 1 ? lut.anchor3b(p) : lut.anchor3c(p);
}
__device__ inline int bc7_anchor(int ns, int p, int s) { return bc7_anchor(ns, p, s, Bc7ConstLut{}); }

// ------------------------------------------------------------- bit access
// A 128-bit block held as two little-endian 64-bit halves.
struct Blk128 {
    uint64_t lo, hi;
};

// Bits pos .. pos + n - 1 of the block (0 <= pos < 128, 1 <= n <= 31):
// a funnel shift of the two halves, without branches (positions differ
// from lane to lane).  (hi << 1) << (63 - p) is hi << (64 - p), zero at p = 0.
__device__ inline uint32_t get_field(const Blk128 &b, int pos, int n)
{
    const int p = pos & 63;
    const uint64_t below = (b.lo >> p) | ((b.hi << 1) << (63 - p));
    const uint64_t v = pos >= 64 ? b.hi >> p : below;
    return (uint32_t)v & ((1u << n) - 1u);
}

// ------------------------------------------------------------- BC1 decode
__device__ inline void bc1_expand(uint32_t c, int e[3])
{
    int r5 = (c >> 11) & 31, g6 = (c >> 5) & 63, b5 = c & 31;
    e[0] = (r5 << 3) | (r5 >> 2);
    e[1] = (g6 << 2) | (g6 >> 4);
    e[2] = (b5 << 3) | (b5 >> 2);
}

// Texel i of a BC1 block given as two 32-bit words; RGBA packed in a uint32
// (R in the low byte).
__device__ inline uint32_t bc1_texel(uint32_t w0, uint32_t w1, int i)
{
    uint32_t c0 = w0 & 0xFFFF, c1 = w0 >> 16;
    int k = (w1 >> (2 * i)) & 3;
    int e0[3], e1[3];
    bc1_expand(c0, e0);
    bc1_expand(c1, e1);
    int px[3];
    uint32_t a = 255;
    if (k == 0) { px[0] = e0[0]; px[1] = e0[1]; px[2] = e0[2]; }
    else if (k == 1) { px[0] = e1[0]; px[1] = e1[1]; px[2] = e1[2]; }
    else if (c0 > c1) {
        for (int c = 0; c < 3; c++)
            px[c] = k == 2 ? (2 * e0[c] + e1[c] + 1) / 3 : (e0[c] + 2 * e1[c] + 1) / 3;
    } else if (k == 2) {
        for (int c = 0; c < 3; c++) px[c] = (e0[c] + e1[c] + 1) >> 1;
    } else {
        px[0] = px[1] = px[2] = 0;
        a = 0;
    }
    return (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) | (a << 24);
}

// ------------------------------------------------------------- BC7 decode
// Texel i of a BC7 block, RGBA packed in a uint32 (R in the low byte).
template <class Lut>
__device__ inline uint32_t bc7_texel(const Blk128 &b, int i, const Lut &lut)
{
    uint32_t b0 = (uint32_t)b.lo & 0xFF;
    if (b0 == 0) return 0;  // reserved mode: all zero
    int m = __ffs(b0) - 1;
    Bc7Mode md = bc7_mode(m);
    int pos = m + 1;
    int part = md.partbits ? (int)get_field(b, pos, md.partbits) : 0;
    pos += md.partbits;
    int rot = md.rotbits ? (int)get_field(b, pos, md.rotbits) : 0;
    pos += md.rotbits;
    int sel = md.selbits ? (int)get_field(b, pos, 1) : 0;
    pos += md.selbits;
    int ns = md.ns, ne = 2 * ns;
    int s = bc7_subset(ns, part, i, lut);
    int e0[4], e1[4];
    int cpos = pos;
    pos += 3 * ne * md.cb;
    int apos = pos;
    pos += ne * md.ab;
    int p0 = 0, p1 = 0;
    if (md.pb == 2) { p0 = (int)get_field(b, pos + 2 * s, 1); p1 = (int)get_field(b, pos + 2 * s + 1, 1); pos += ne; }
    else if (md.pb == 1) { p0 = p1 = (int)get_field(b, pos + s, 1); pos += ns; }
    int nbits = md.cb + (md.pb ? 1 : 0);
    for (int c = 0; c < 3; c++) {
        int v0 = (int)get_field(b, cpos + (c * ne + 2 * s) * md.cb, md.cb);
        int v1 = (int)get_field(b, cpos + (c * ne + 2 * s + 1) * md.cb, md.cb);
        if (md.pb) { v0 = (v0 << 1) | p0; v1 = (v1 << 1) | p1; }
        e0[c] = expand_bits(v0, nbits);
        e1[c] = expand_bits(v1, nbits);
    }
    if (md.ab) {
        int abits = md.ab + (md.pb ? 1 : 0);
        int v0 = (int)get_field(b, apos + 2 * s * md.ab, md.ab);
        int v1 = (int)get_field(b, apos + (2 * s + 1) * md.ab, md.ab);
        if (md.pb) { v0 = (v0 << 1) | p0; v1 = (v1 << 1) | p1; }
        e0[3] = expand_bits(v0, abits);
        e1[3] = expand_bits(v1, abits);
    } else {
        e0[3] = e1[3] = 255;
    }
    // primary index: one bit less for each anchor texel before i and for i itself
    int a1 = ns >= 2 ? bc7_anchor(ns, part, 1, lut) : 99;
    int a2 = ns == 3 ? bc7_anchor(ns, part, 2, lut) : 99;
    int before = (i > 0) + (a1 < i) + (a2 < i);
    int anchored = (i == 0) || (i == a1) || (i == a2);
    int i1 = (int)get_field(b, pos + i * md.ib - before, md.ib - anchored);
    pos += 16 * md.ib - ns;
    int i2 = 0;
    if (md.ib2) i2 = (int)get_field(b, pos + i * md.ib2 - (i > 0), md.ib2 - (i == 0));
    int ci = i1, cn = md.ib, ai = i1, an = md.ib;
    if (md.ib2) {
        if (sel == 0) { ai = i2; an = md.ib2; }
        else { ci = i2; cn = md.ib2; ai = i1; an = md.ib; }
    }
    int wc = bc7_weight_packed(cn, ci), wa = bc7_weight_packed(an, ai);
    int px[4];
    for (int c = 0; c < 3; c++) px[c] = interp64(e0[c], e1[c], wc);
    px[3] = interp64(e0[3], e1[3], wa);
    if (rot) { int t = px[3]; px[3] = px[rot - 1]; px[rot - 1] = t; }
    return (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) | ((uint32_t)px[3] << 24);
}
__device__ inline uint32_t bc7_texel(const Blk128 &b, int i) { return bc7_texel(b, i, Bc7ConstLut{}); }

}  // namespace gsbc
