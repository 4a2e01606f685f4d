// BC6H block unpacking for the decode kernels (gfx950).
//
// Implements the BC6H format definition that Section 4.2 of the paper
// ("Trainable BC6 decompression") defers to, in its exact integer form:
// endpoint unquantisation (the integer form of eq. 6), weighted blending of
// the two endpoints of the texel's subset (eq. 7), and the scale by 31/64
// (unsigned) or 31/32 (signed) whose result is reinterpreted as a half
// (eq. 8).
//
// Layout strategy (branch-free across lanes holding different modes):
//  * In every two-subset mode the main runs of the header fields sit at the
//    same block positions: w at 5/15/25, x at 35/45/55, gy[3:0] at 41,
//    gz[3:0] at 51, by[3:0] at 61, ry at 65, rz at 71, partition at 77.
//    Only their lengths change with the mode.
//  * The remaining header bits are single "extra" bits (gy4, gy5, by4, by5,
//    gz4, gz5, bz0..bz5 and bit 10 of w) whose positions a small per-mode
//    table lists.
//  * One-subset modes store x in the 10-bit chunks at 35/45/55 and the
//    endpoint bits above 10 of w reversed at the top of those chunks.
// So one instruction stream decodes all 14 modes.
//
// Everything here is __host__ __device__ so the same code can be exercised
// on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcf {

// ---------------------------------------------------------------------------
// bit helpers (the device compiler maps them to v_bfe / v_alignbit / v_bfrev)

__host__ __device__ __forceinline__ uint32_t ubits(uint32_t x, uint32_t off, uint32_t len)
{
    return len ? (x >> off) & (0xFFFFFFFFu >> (32u - len)) : 0u;
}

__host__ __device__ __forceinline__ int32_t sext(uint32_t x, uint32_t len)
{
    // sign-extend the low `len` (1..32) bits
    const uint32_t s = 32u - len;
    return (int32_t)(x << s) >> s;
}

__host__ __device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

// lo | hi << 16 for 16-bit lo and hi. On the GPU one byte permute: written as
// a shift, the compiler folds the shift into the multiply that produced hi,
// turning a full-rate 24-bit multiply into a quarter-rate 32-bit one.
__host__ __device__ __forceinline__ uint32_t pack_lo_hi(uint32_t lo, uint32_t hi)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
#else
    return (lo & 0xFFFFu) | (hi << 16);
#endif
}

// reverse the low k bits of v (k = 0..32)
__host__ __device__ __forceinline__ uint32_t reverse_low(uint32_t v, uint32_t k)
{
    return (uint32_t)((uint64_t)__builtin_bitreverse32(v) >> (32u - k));
}

// ---------------------------------------------------------------------------
// per-mode descriptors

// word 0: [0] valid [1] two subsets [2] transformed [3..7] endpoint bits
//         [8..11] delta bits r [12..15] g [16..19] b
//         [20..23] one-subset modes: w bits above 10 stored reversed in x's chunk
// words 1..4: extra bits, one byte each, 0x80 | block position, 0 = absent:
//         gy4 gy5 by4 by5 | gz4 gz5 bz0 bz1 | bz2 bz3 bz4 bz5 | rw10 gw10 bw10 -
constexpr int kModeWords = 5;
constexpr int kModes = 15;                 // row 0: reserved codes
constexpr int kPartitions = 32;
constexpr int kTableWords = kModes * kModeWords + kPartitions;

#define BCF_INFO(two, tr, eb, dr, dg, db, kh)                                                 \
    (1u | ((uint32_t)(two) << 1) | ((uint32_t)(tr) << 2) | ((uint32_t)(eb) << 3) |          \
     ((uint32_t)(dr) << 8) | ((uint32_t)(dg) << 12) | ((uint32_t)(db) << 16) |               \
     ((uint32_t)(kh) << 20))
#define BCF_AT(p) (0x80u | (uint32_t)(p))
#define BCF_BYTES(a, b, c, d)                                                                 \
    ((uint32_t)(a) | ((uint32_t)(b) << 8) | ((uint32_t)(c) << 16) | ((uint32_t)(d) << 24))

// mode rows, then per partition: subset-1 mask (bit t: texel t) | anchor << 16
static constexpr uint32_t kTable[kTableWords] = {
    // reserved
    0, 0, 0, 0, 0,
    // 1: 10-bit w, deltas 5/5/5
    BCF_INFO(1, 1, 10, 5, 5, 5, 0),
    BCF_BYTES(BCF_AT(2), 0, BCF_AT(3), 0), BCF_BYTES(BCF_AT(40), 0, BCF_AT(50), BCF_AT(60)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), BCF_AT(4), 0), 0,
    // 2: 7-bit w, deltas 6/6/6
    BCF_INFO(1, 1, 7, 6, 6, 6, 0),
    BCF_BYTES(BCF_AT(24), BCF_AT(2), BCF_AT(14), BCF_AT(22)),
    BCF_BYTES(BCF_AT(3), BCF_AT(4), BCF_AT(12), BCF_AT(13)),
    BCF_BYTES(BCF_AT(23), BCF_AT(32), BCF_AT(34), BCF_AT(33)), 0,
    // 3: 11-bit w, deltas 5/4/4
    BCF_INFO(1, 1, 11, 5, 4, 4, 0),
    0, BCF_BYTES(0, 0, BCF_AT(50), BCF_AT(60)), BCF_BYTES(BCF_AT(70), BCF_AT(76), 0, 0),
    BCF_BYTES(BCF_AT(40), BCF_AT(49), BCF_AT(59), 0),
    // 4: 11-bit w, deltas 4/5/4
    BCF_INFO(1, 1, 11, 4, 5, 4, 0),
    BCF_BYTES(BCF_AT(75), 0, 0, 0), BCF_BYTES(BCF_AT(40), 0, BCF_AT(69), BCF_AT(60)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), 0, 0), BCF_BYTES(BCF_AT(39), BCF_AT(50), BCF_AT(59), 0),
    // 5: 11-bit w, deltas 4/4/5
    BCF_INFO(1, 1, 11, 4, 4, 5, 0),
    BCF_BYTES(0, 0, BCF_AT(40), 0), BCF_BYTES(0, 0, BCF_AT(50), BCF_AT(69)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), BCF_AT(75), 0), BCF_BYTES(BCF_AT(39), BCF_AT(49), BCF_AT(60), 0),
    // 6: 9-bit w, deltas 5/5/5
    BCF_INFO(1, 1, 9, 5, 5, 5, 0),
    BCF_BYTES(BCF_AT(24), 0, BCF_AT(14), 0), BCF_BYTES(BCF_AT(40), 0, BCF_AT(50), BCF_AT(60)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), BCF_AT(34), 0), 0,
    // 7: 8-bit w, deltas 6/5/5
    BCF_INFO(1, 1, 8, 6, 5, 5, 0),
    BCF_BYTES(BCF_AT(24), 0, BCF_AT(14), 0), BCF_BYTES(BCF_AT(13), 0, BCF_AT(50), BCF_AT(60)),
    BCF_BYTES(BCF_AT(23), BCF_AT(33), BCF_AT(34), 0), 0,
    // 8: 8-bit w, deltas 5/6/5
    BCF_INFO(1, 1, 8, 5, 6, 5, 0),
    BCF_BYTES(BCF_AT(24), BCF_AT(23), BCF_AT(14), 0),
    BCF_BYTES(BCF_AT(40), BCF_AT(33), BCF_AT(13), BCF_AT(60)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), BCF_AT(34), 0), 0,
    // 9: 8-bit w, deltas 5/5/6
    BCF_INFO(1, 1, 8, 5, 5, 6, 0),
    BCF_BYTES(BCF_AT(24), 0, BCF_AT(14), BCF_AT(23)),
    BCF_BYTES(BCF_AT(40), 0, BCF_AT(50), BCF_AT(13)),
    BCF_BYTES(BCF_AT(70), BCF_AT(76), BCF_AT(34), BCF_AT(33)), 0,
    // 10: four untransformed 6-bit endpoints
    BCF_INFO(1, 0, 6, 6, 6, 6, 0),
    BCF_BYTES(BCF_AT(24), BCF_AT(21), BCF_AT(14), BCF_AT(22)),
    BCF_BYTES(BCF_AT(11), BCF_AT(31), BCF_AT(12), BCF_AT(13)),
    BCF_BYTES(BCF_AT(23), BCF_AT(32), BCF_AT(34), BCF_AT(33)), 0,
    // 11..14: one subset; x in the 10-bit chunks, top kh bits of a chunk = w[10..] reversed
    BCF_INFO(0, 0, 10, 10, 10, 10, 0), 0, 0, 0, 0,
    BCF_INFO(0, 1, 11, 9, 9, 9, 1), 0, 0, 0, 0,
    BCF_INFO(0, 1, 12, 8, 8, 8, 2), 0, 0, 0, 0,
    BCF_INFO(0, 1, 16, 4, 4, 4, 6), 0, 0, 0, 0,
    // partitions
    0xCCCCu | 15u << 16, 0x8888u | 15u << 16, 0xEEEEu | 15u << 16, 0xECC8u | 15u << 16,
    0xC880u | 15u << 16, 0xFEECu | 15u << 16, 0xFEC8u | 15u << 16, 0xEC80u | 15u << 16,
    0xC800u | 15u << 16, 0xFFECu | 15u << 16, 0xFE80u | 15u << 16, 0xE800u | 15u << 16,
    0xFFE8u | 15u << 16, 0xFF00u | 15u << 16, 0xFFF0u | 15u << 16, 0xF000u | 15u << 16,
    0xF710u | 15u << 16, 0x008Eu | 2u << 16,  0x7100u | 8u << 16,  0x08CEu | 2u << 16,
    0x008Cu | 2u << 16,  0x7310u | 8u << 16,  0x3100u | 8u << 16,  0x8CCEu | 15u << 16,
    0x088Cu | 2u << 16,  0x3110u | 8u << 16,  0x6666u | 2u << 16,  0x366Cu | 2u << 16,
    0x17E8u | 8u << 16,  0x0FF0u | 8u << 16,  0x718Eu | 2u << 16,  0x399Cu | 2u << 16,
};

#undef BCF_INFO
#undef BCF_AT
#undef BCF_BYTES

// Mode number (1..14, 0 = reserved) for each value of the low five bits: two
// bits 00/01 select modes 1/2 whatever follows; otherwise all five bits count.
__host__ __device__ __forceinline__ uint32_t mode_of(uint32_t d0)
{
    const uint32_t code = d0 & 31u;
    const uint64_t lut = code < 16 ? 0xE621D521C421B321ull : 0x0A21092108210721ull;
    return (uint32_t)(lut >> ((code & 15u) * 4u)) & 15u;
}

// ---------------------------------------------------------------------------
// unpacked header: for subset s and channel c the texel value before the final
// scale is (base[s][c] + w * diff[s][c]) >> 6, w = weight of the texel's index

struct Bc6hHeader {
    int32_t base[2][3];      // 64 * first endpoint + 32
    int32_t diff[2][3];      // second endpoint - first endpoint
    uint32_t mask;           // texels in subset 1 (0 for one-subset modes)
    uint64_t idx;            // texel t's index at bits [ib*t, ib*t+ib)
    uint32_t ib;             // index bits per texel: 3 or 4
    uint32_t valid;
};

template <bool SIGNED>
__host__ __device__ __forceinline__ int32_t unquantize(int32_t e, uint32_t eb)
{
    if (!SIGNED) {
        // ((e << 16) + 2^15) >> eb; 0 and the top code map to 0 and 0xFFFF.
        // For eb = 16 the general expression already returns e.
        uint32_t u = (((uint32_t)e << 16) | 0x8000u) >> eb;
        u = e == 0 ? 0u : u;
        u = (uint32_t)e == (0xFFFFFFFFu >> (32u - eb)) ? 0xFFFFu : u;
        return (int32_t)u;
    } else {
        const uint32_t m = (uint32_t)(e < 0 ? -e : e);
        uint32_t u = ((m << 15) | 0x4000u) >> (eb - 1u);
        u = m == 0 ? 0u : u;
        u = m >= ((1u << (eb - 1u)) - 1u) ? 0x7FFFu : u;
        int32_t r = e < 0 ? -(int32_t)u : (int32_t)u;
        return eb >= 16u ? e : r;
    }
}

template <bool SIGNED>
__host__ __device__ __forceinline__ void bc6h_header(uint32_t d0, uint32_t d1, uint32_t d2,
                                                     uint32_t d3, const uint32_t *table,
                                                     Bc6hHeader &h)
{
    const uint32_t mode = mode_of(d0);
    const uint32_t *md = table + kModeWords * mode;
    const uint32_t info = md[0];
    const uint32_t x0 = md[1], x1 = md[2], x2 = md[3], x3 = md[4];
    const uint32_t two = (info >> 1) & 1u;
    const uint32_t transformed = (info >> 2) & 1u;
    const uint32_t eb = (info >> 3) & 31u;
    const uint32_t dr = (info >> 8) & 15u, dg = (info >> 12) & 15u, db = (info >> 16) & 15u;
    const uint32_t kh = (info >> 20) & 15u;
    h.valid = info & 1u;

    auto extra = [&](uint32_t word, uint32_t slot) -> uint32_t {
        const uint32_t e = (word >> (8u * slot)) & 255u;
        const uint32_t pos = e & 127u;
        const uint32_t src = pos < 32u ? d0 : (pos < 64u ? d1 : d2);
        return (src >> (pos & 31u)) & (e >> 7);
    };

    // w: low min(eb,10) bits at 5/15/25
    const uint32_t wlen = eb < 10u ? eb : 10u;
    uint32_t w[3];
    w[0] = ubits(d0, 5, wlen);
    w[1] = ubits(d0, 15, wlen);
    w[2] = ubits(funnel(d1, d0, 25), 0, wlen);
    // 10-bit chunks at 35/45/55 hold x (low delta bits)
    const uint32_t chunk[3] = {ubits(d1, 3, 10), ubits(d1, 13, 10), ubits(funnel(d2, d1, 23), 0, 10)};
    const uint32_t dw[3] = {dr, dg, db};
    // w bits above 10: one extra bit in two-subset modes, the top kh bits of
    // the chunk, reversed, in one-subset modes
    for (int c = 0; c < 3; ++c) {
        const uint32_t hi = two ? extra(x3, (uint32_t)c) : reverse_low(chunk[c] >> dw[c], kh);
        w[c] |= hi << 10;
    }
    uint32_t f[3][3];    // stored x, y, z per channel
    for (int c = 0; c < 3; ++c) f[0][c] = ubits(chunk[c], 0, dw[c]);
    f[1][0] = ubits(d2, 1, dr);                                                  // ry at 65
    f[1][1] = ubits(d1, 9, 4) | extra(x0, 0) << 4 | extra(x0, 1) << 5;          // gy[3:0] at 41
    f[1][2] = ubits(funnel(d2, d1, 29), 0, 4) | extra(x0, 2) << 4 | extra(x0, 3) << 5;  // by at 61
    f[2][0] = ubits(d2, 7, dr);                                                  // rz at 71
    f[2][1] = ubits(d1, 19, 4) | extra(x1, 0) << 4 | extra(x1, 1) << 5;         // gz[3:0] at 51
    f[2][2] = extra(x1, 2) | extra(x1, 3) << 1 | extra(x2, 0) << 2 | extra(x2, 1) << 3 |
              extra(x2, 2) << 4 | extra(x2, 3) << 5;
    const uint32_t part = ubits(d2, 13, 5);

    // endpoints: x, y, z are deltas from w in transformed modes
    const uint32_t emask = 0xFFFFFFFFu >> (32u - (eb ? eb : 1u));
    int32_t e[4][3];
    for (int c = 0; c < 3; ++c) {
        e[0][c] = SIGNED ? sext(w[c], eb ? eb : 1u) : (int32_t)w[c];
        for (int j = 0; j < 3; ++j) {
            uint32_t v = transformed ? (uint32_t)((int32_t)w[c] + sext(f[j][c], dw[c] ? dw[c] : 1u))
                                     : f[j][c];
            v &= emask;
            e[j + 1][c] = SIGNED ? sext(v, eb ? eb : 1u) : (int32_t)v;
        }
    }
    const uint32_t ebq = eb ? eb : 16u;      // reserved rows: any valid shift
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 3; ++c) {
            const int32_t a = unquantize<SIGNED>(e[2 * s][c], ebq);
            const int32_t b = unquantize<SIGNED>(e[2 * s + 1][c], ebq);
            h.base[s][c] = 64 * a + 32;
            h.diff[s][c] = b - a;
        }

    // indices: give every texel the full index width by re-inserting the
    // implicit zero top bit of texel 0 and of the subset-1 anchor
    const uint32_t pinfo = table[kModes * kModeWords + part];
    uint64_t idx;
    if (two) {
        const uint32_t anchor = pinfo >> 16;
        idx = (((uint64_t)d3 << 32) | d2) >> 18;                                 // bits 82..127
        idx = ((idx >> 2) << 3) | (idx & 3u);
        const uint32_t p = 3u * anchor + 2u;
        idx = ((idx >> p) << (p + 1u)) | (idx & ((1ull << p) - 1u));
        h.mask = pinfo & 0xFFFFu;
        h.ib = 3;
    } else {
        idx = (((uint64_t)d3 << 32) | d2) >> 1;                                  // bits 65..127
        idx = ((idx >> 3) << 4) | (idx & 7u);
        h.mask = 0;
        h.ib = 4;
    }
    h.idx = idx;
}

// Half bit pattern of texel t (0..15), channel c. Weights are the format's
// round(64 i / 7) and round(64 i / 15), computed as (i * 585 + 32) >> 6 and
// (i * 273 + 32) >> 6.
template <bool SIGNED>
__host__ __device__ __forceinline__ uint32_t bc6h_texel(const Bc6hHeader &h, uint32_t t, int c)
{
    // operands masked to their known widths (no-ops here) so the compiler can
    // use the full-rate 24-bit multiplies
    const uint32_t i = (uint32_t)(h.idx >> (h.ib * t)) & ((1u << h.ib) - 1u) & 15u;
    const uint32_t wt = (i * (h.ib == 3 ? 585u : 273u) + 32u) >> 6;
    const uint32_t s = (h.mask >> t) & 1u;
    const int32_t base = s ? h.base[1][c] : h.base[0][c];
    // |diff| < 2^17 and wt <= 64
    const int32_t diff = (int32_t)((uint32_t)(s ? h.diff[1][c] : h.diff[0][c]) << 8) >> 8;
    const int32_t v = (base + (int32_t)(wt & 127u) * diff) >> 6;   // arithmetic: floor
    uint32_t out;
    if (!SIGNED) {
        out = (((uint32_t)v & 0xFFFFFFu) * 31u) >> 6;                 // v <= 0xFFFF
    } else {
        const uint32_t m = (uint32_t)(v < 0 ? -v : v);
        out = (((m & 0xFFFFFFu) * 31u) >> 5) | (v < 0 ? 0x8000u : 0u); // |v| <= 0x7FFF
    }
    return h.valid ? out : 0u;
}

// The at most 16 distinct values a block's texels take, channels packed as
// (r | g << 16, b): entry j = 8 s + i for two-subset modes (3-bit index i of
// subset s), j = i for one-subset modes (4-bit index i). Each entry is the
// blend and finish of bc6h_texel for that subset and index.
template <bool SIGNED>
__host__ __device__ __forceinline__ void bc6h_palette(const Bc6hHeader &h, uint32_t pal[16][2])
{
    const bool two = h.ib == 3;
    // entries 0..7 blend subset 0; entries 8..15 subset 1 (two subsets) or
    // subset 0 again (one subset). A reserved mode decodes to zeros: base and
    // diff 0 give v = 0. |diff| < 2^17 and wt <= 64, so the products fit the
    // 24-bit multiply once diff is restated as a 24-bit value.
    int32_t b_lo[3], d_lo[3], b_hi[3], d_hi[3];
    for (int c = 0; c < 3; ++c) {
        const int32_t db0 = (int32_t)((uint32_t)h.diff[0][c] << 8) >> 8;
        const int32_t db1 = (int32_t)((uint32_t)h.diff[1][c] << 8) >> 8;
        b_lo[c] = h.valid ? h.base[0][c] : 0;
        d_lo[c] = h.valid ? db0 : 0;
        b_hi[c] = h.valid ? (two ? h.base[1][c] : h.base[0][c]) : 0;
        d_hi[c] = h.valid ? (two ? db1 : db0) : 0;
    }
#pragma unroll
    for (uint32_t j = 0; j < 16; ++j) {
        const int32_t wt = (int32_t)(two ? (((j & 7u) * 585u + 32u) >> 6) : ((j * 273u + 32u) >> 6));
        uint32_t ch[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int32_t v = ((j < 8 ? b_lo[c] : b_hi[c]) + wt * (j < 8 ? d_lo[c] : d_hi[c])) >> 6;
            if (!SIGNED) {
                ch[c] = (((uint32_t)v & 0xFFFFFFu) * 31u) >> 6;                      // v <= 0xFFFF
            } else {
                const uint32_t m = (uint32_t)(v < 0 ? -v : v);
                ch[c] = (((m & 0xFFFFFFu) * 31u) >> 5) | (v < 0 ? 0x8000u : 0u);    // |v| <= 0x7FFF
            }
        }
        pal[j][0] = pack_lo_hi(ch[0], ch[1]);
        pal[j][1] = ch[2];
    }
}

// Palette entry of texel t (0..15).
__host__ __device__ __forceinline__ uint32_t bc6h_slot(const Bc6hHeader &h, uint32_t t)
{
    const uint32_t i = (uint32_t)(h.idx >> (h.ib * t)) & ((1u << h.ib) - 1u);
    return h.ib == 3 ? ((((h.mask >> t) & 1u) << 3) | i) : i;
}

// Eight 3-bit fields (bits 3k..3k+2 of x) moved to 4-bit nibbles (bits 4k..4k+2).
__host__ __device__ __forceinline__ uint32_t spread3to4(uint32_t x)
{
    x = (x & 0x00000FFFu) | ((x & 0x00FFF000u) << 4);      // fields 4..7 up by 4
    x = (x & 0x003F003Fu) | ((x & 0x0FC00FC0u) << 2);      // fields 2, 3, 6, 7 up by 2
    return (x & 0x07070707u) | ((x & 0x38383838u) << 1);   // fields 1, 3, 5, 7 up by 1
}

// Eight bits (bit k of x) moved to bit 4k.
__host__ __device__ __forceinline__ uint32_t spread1to4(uint32_t x)
{
    x = (x & 0x0000000Fu) | ((x & 0x000000F0u) << 12);     // bits 4..7 to 16..19
    x = (x & 0x00030003u) | ((x & 0x000C000Cu) << 6);      // bits 2, 3 (18, 19) up by 6
    return (x & 0x01010101u) | ((x & 0x02020202u) << 3);   // bits 1 (9, 17, 25) up by 3
}

// Palette entries of all 16 texels, four bits each: texel t's bc6h_slot at
// bits 4t..4t+3 of s0 (t < 8) or s1 (t >= 8).
__host__ __device__ __forceinline__ void bc6h_slots(const Bc6hHeader &h, uint32_t &s0, uint32_t &s1)
{
    if (h.ib == 4) {                          // one subset: the 4-bit indices are the slots
        s0 = (uint32_t)h.idx;
        s1 = (uint32_t)(h.idx >> 32);
    } else {                                  // two subsets: 3-bit index | subset << 3
        s0 = spread3to4((uint32_t)h.idx & 0xFFFFFFu) | (spread1to4(h.mask & 0xFFu) << 3);
        s1 = spread3to4((uint32_t)(h.idx >> 24) & 0xFFFFFFu) | (spread1to4((h.mask >> 8) & 0xFFu) << 3);
    }
}

}  // namespace bcf
