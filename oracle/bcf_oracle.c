/*
 * bcf_oracle.c -- plain CPU oracle for block-compressed neural material decode
 * (Weinreich et al., "Real-Time Neural Materials using Block-Compressed
 * Features", arXiv 2311.16121).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg are its only users. It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes, in the paper's order:
 *   1. BC6H decode of a block to half-float texels. The paper defers the layout
 *      to the DirectX BC6H definition (Section "Block parameterization"); the
 *      arithmetic is its eqs. (6)-(8) in the format's exact integer form.
 *   2. Trilinear filtering of each feature pyramid, eq. (9), at the per-texture
 *      scale s_i = s + b_i of eq. (10).
 *   3. Concatenation of the filtered features and the decoder MLP f_eta, eq. (3).
 *
 * Written for obviousness, not speed: every texel tap decodes its whole block
 * again, and everything after the integer decode is binary64.
 */
#include "bcf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* IEEE 754 binary16 -> binary64 (IEEE 754-2008, binary16 interchange format) */

double bcfo_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int exponent = (h >> 10) & 0x1F;
    int mantissa = h & 0x3FF;
    double value;
    if (exponent == 0)                       /* zero and subnormals */
        value = ldexp((double)mantissa, -24);
    else if (exponent == 31)                 /* infinities and NaNs */
        value = mantissa ? NAN : INFINITY;
    else                                     /* normal numbers */
        value = ldexp(1024.0 + mantissa, exponent - 25);
    return sign ? -value : value;
}

/* ------------------------------------------------------------------------ */
/* BC6H layout, transcribed from the public BC6H format definition.
 *
 * Each mode lists its header fields from block bit 0 upward in the
 * definition's own notation f[a:b]: the run occupies |a-b|+1 consecutive
 * block bits, the lowest of which holds field bit b, stepping towards a.
 * So rw[9:0] stores rw bit 0 first, and rw[10:15] stores rw bit 15 first.
 * Fields: m = mode code, d = partition, w/x/y/z = the four endpoints
 * (x, y, z are deltas from w in transformed modes), r/g/b = channel. */

enum { F_M, F_D, F_RW, F_GW, F_BW, F_RX, F_GX, F_BX, F_RY, F_GY, F_BY, F_RZ, F_GZ, F_BZ, F_COUNT };

typedef struct { unsigned char f, a, b; } run_t;

typedef struct {
    unsigned code, code_bits;   /* mode code value and its width */
    int regions;                /* 1 or 2 subsets */
    int transformed;            /* endpoints x,y,z stored as deltas from w */
    int ep_bits;                /* endpoint precision */
    int delta_bits[3];          /* stored width of x, y, z per channel */
    run_t runs[40];             /* ends at the first all-zero entry */
} mode_t;

#define R(f, a, b) { F_##f, a, b }

static const mode_t MODES[14] = {
    /* mode 1 */
    { 0x00, 2, 2, 1, 10, {5, 5, 5}, {
        R(M,1,0), R(GY,4,4), R(BY,4,4), R(BZ,4,4), R(RW,9,0), R(GW,9,0), R(BW,9,0),
        R(RX,4,0), R(GZ,4,4), R(GY,3,0), R(GX,4,0), R(BZ,0,0), R(GZ,3,0), R(BX,4,0),
        R(BZ,1,1), R(BY,3,0), R(RY,4,0), R(BZ,2,2), R(RZ,4,0), R(BZ,3,3), R(D,4,0) } },
    /* mode 2 */
    { 0x01, 2, 2, 1, 7, {6, 6, 6}, {
        R(M,1,0), R(GY,5,5), R(GZ,4,4), R(GZ,5,5), R(RW,6,0), R(BZ,0,0), R(BZ,1,1),
        R(BY,4,4), R(GW,6,0), R(BY,5,5), R(BZ,2,2), R(GY,4,4), R(BW,6,0), R(BZ,3,3),
        R(BZ,5,5), R(BZ,4,4), R(RX,5,0), R(GY,3,0), R(GX,5,0), R(GZ,3,0), R(BX,5,0),
        R(BY,3,0), R(RY,5,0), R(RZ,5,0), R(D,4,0) } },
    /* mode 3 */
    { 0x02, 5, 2, 1, 11, {5, 4, 4}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,4,0), R(RW,10,10), R(GY,3,0),
        R(GX,3,0), R(GW,10,10), R(BZ,0,0), R(GZ,3,0), R(BX,3,0), R(BW,10,10), R(BZ,1,1),
        R(BY,3,0), R(RY,4,0), R(BZ,2,2), R(RZ,4,0), R(BZ,3,3), R(D,4,0) } },
    /* mode 4 */
    { 0x06, 5, 2, 1, 11, {4, 5, 4}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,3,0), R(RW,10,10), R(GZ,4,4),
        R(GY,3,0), R(GX,4,0), R(GW,10,10), R(GZ,3,0), R(BX,3,0), R(BW,10,10), R(BZ,1,1),
        R(BY,3,0), R(RY,3,0), R(BZ,0,0), R(BZ,2,2), R(RZ,3,0), R(GY,4,4), R(BZ,3,3),
        R(D,4,0) } },
    /* mode 5 */
    { 0x0A, 5, 2, 1, 11, {4, 4, 5}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,3,0), R(RW,10,10), R(BY,4,4),
        R(GY,3,0), R(GX,3,0), R(GW,10,10), R(BZ,0,0), R(GZ,3,0), R(BX,4,0), R(BW,10,10),
        R(BY,3,0), R(RY,3,0), R(BZ,1,1), R(BZ,2,2), R(RZ,3,0), R(BZ,4,4), R(BZ,3,3),
        R(D,4,0) } },
    /* mode 6 */
    { 0x0E, 5, 2, 1, 9, {5, 5, 5}, {
        R(M,4,0), R(RW,8,0), R(BY,4,4), R(GW,8,0), R(GY,4,4), R(BW,8,0), R(BZ,4,4),
        R(RX,4,0), R(GZ,4,4), R(GY,3,0), R(GX,4,0), R(BZ,0,0), R(GZ,3,0), R(BX,4,0),
        R(BZ,1,1), R(BY,3,0), R(RY,4,0), R(BZ,2,2), R(RZ,4,0), R(BZ,3,3), R(D,4,0) } },
    /* mode 7 */
    { 0x12, 5, 2, 1, 8, {6, 5, 5}, {
        R(M,4,0), R(RW,7,0), R(GZ,4,4), R(BY,4,4), R(GW,7,0), R(BZ,2,2), R(GY,4,4),
        R(BW,7,0), R(BZ,3,3), R(BZ,4,4), R(RX,5,0), R(GY,3,0), R(GX,4,0), R(BZ,0,0),
        R(GZ,3,0), R(BX,4,0), R(BZ,1,1), R(BY,3,0), R(RY,5,0), R(RZ,5,0), R(D,4,0) } },
    /* mode 8 */
    { 0x16, 5, 2, 1, 8, {5, 6, 5}, {
        R(M,4,0), R(RW,7,0), R(BZ,0,0), R(BY,4,4), R(GW,7,0), R(GY,5,5), R(GY,4,4),
        R(BW,7,0), R(GZ,5,5), R(BZ,4,4), R(RX,4,0), R(GZ,4,4), R(GY,3,0), R(GX,5,0),
        R(GZ,3,0), R(BX,4,0), R(BZ,1,1), R(BY,3,0), R(RY,4,0), R(BZ,2,2), R(RZ,4,0),
        R(BZ,3,3), R(D,4,0) } },
    /* mode 9 */
    { 0x1A, 5, 2, 1, 8, {5, 5, 6}, {
        R(M,4,0), R(RW,7,0), R(BZ,1,1), R(BY,4,4), R(GW,7,0), R(BY,5,5), R(GY,4,4),
        R(BW,7,0), R(BZ,5,5), R(BZ,4,4), R(RX,4,0), R(GZ,4,4), R(GY,3,0), R(GX,4,0),
        R(BZ,0,0), R(GZ,3,0), R(BX,5,0), R(BY,3,0), R(RY,4,0), R(BZ,2,2), R(RZ,4,0),
        R(BZ,3,3), R(D,4,0) } },
    /* mode 10: two subsets, four untransformed 6-bit endpoints */
    { 0x1E, 5, 2, 0, 6, {6, 6, 6}, {
        R(M,4,0), R(RW,5,0), R(GZ,4,4), R(BZ,0,0), R(BZ,1,1), R(BY,4,4), R(GW,5,0),
        R(GY,5,5), R(BY,5,5), R(BZ,2,2), R(GY,4,4), R(BW,5,0), R(GZ,5,5), R(BZ,3,3),
        R(BZ,5,5), R(BZ,4,4), R(RX,5,0), R(GY,3,0), R(GX,5,0), R(GZ,3,0), R(BX,5,0),
        R(BY,3,0), R(RY,5,0), R(RZ,5,0), R(D,4,0) } },
    /* mode 11: one subset, two untransformed 10-bit endpoints */
    { 0x03, 5, 1, 0, 10, {10, 10, 10}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,9,0), R(GX,9,0), R(BX,9,0) } },
    /* mode 12 */
    { 0x07, 5, 1, 1, 11, {9, 9, 9}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,8,0), R(RW,10,10), R(GX,8,0),
        R(GW,10,10), R(BX,8,0), R(BW,10,10) } },
    /* mode 13 */
    { 0x0B, 5, 1, 1, 12, {8, 8, 8}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,7,0), R(RW,10,11), R(GX,7,0),
        R(GW,10,11), R(BX,7,0), R(BW,10,11) } },
    /* mode 14 */
    { 0x0F, 5, 1, 1, 16, {4, 4, 4}, {
        R(M,4,0), R(RW,9,0), R(GW,9,0), R(BW,9,0), R(RX,3,0), R(RW,10,15), R(GX,3,0),
        R(GW,10,15), R(BX,3,0), R(BW,10,15) } },
};

#undef R

/* The 32 two-subset partitions P_k (bit t set: texel t is in subset 1) and the
 * texel of subset 1 whose index drops its top bit (its "anchor"), as the
 * format definition lists them. Subset 0's anchor is always texel 0. */
static const uint16_t PARTITION_MASK[32] = {
    0xCCCC, 0x8888, 0xEEEE, 0xECC8, 0xC880, 0xFEEC, 0xFEC8, 0xEC80,
    0xC800, 0xFFEC, 0xFE80, 0xE800, 0xFFE8, 0xFF00, 0xFFF0, 0xF000,
    0xF710, 0x008E, 0x7100, 0x08CE, 0x008C, 0x7310, 0x3100, 0x8CCE,
    0x088C, 0x3110, 0x6666, 0x366C, 0x17E8, 0x0FF0, 0x718E, 0x399C,
};
static const uint8_t PARTITION_ANCHOR[32] = {
    15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
    15,  2,  8,  2,  2,  8,  8, 15,  2,  8,  2,  2,  8,  8,  2,  2,
};

/* Interpolation weights out of 64 for 3- and 4-bit indices. */
static const int WEIGHTS3[8] = {0, 9, 18, 27, 37, 46, 55, 64};
static const int WEIGHTS4[16] = {0, 4, 9, 13, 17, 21, 26, 30, 34, 38, 43, 47, 51, 55, 60, 64};

static unsigned block_bit(const uint8_t *blk, int p)
{
    return (blk[p >> 3] >> (p & 7)) & 1u;
}

static unsigned block_bits(const uint8_t *blk, int p, int n)
{
    unsigned v = 0;
    for (int i = 0; i < n; i++)
        v |= block_bit(blk, p + i) << i;
    return v;
}

static int run_count(const mode_t *md)
{
    int n = 0;
    while (n < 40 && (md->runs[n].f || md->runs[n].a || md->runs[n].b))
        n++;
    return n;
}

/* Mode code: two bits when they read 00 or 01, otherwise five bits. */
static const mode_t *find_mode(const uint8_t *blk, int *mode_number)
{
    unsigned low2 = block_bits(blk, 0, 2);
    unsigned code = low2 < 2 ? low2 : block_bits(blk, 0, 5);
    unsigned width = low2 < 2 ? 2 : 5;
    for (int i = 0; i < 14; i++)
        if (MODES[i].code == code && MODES[i].code_bits == width) {
            *mode_number = i + 1;
            return &MODES[i];
        }
    *mode_number = 0;
    return NULL;
}

/* Walk the mode's runs from bit 0 and assemble every field. Returns the bit
 * position after the header. */
static int read_fields(const uint8_t *blk, const mode_t *md, int32_t field[F_COUNT])
{
    memset(field, 0, sizeof(int32_t) * F_COUNT);
    int p = 0;
    for (int r = 0, n = run_count(md); r < n; r++) {
        const run_t *run = &md->runs[r];
        int step = run->a >= run->b ? 1 : -1;
        for (int k = run->b;; k += step) {
            field[run->f] |= (int32_t)(block_bit(blk, p) << k);
            p++;
            if (k == run->a)
                break;
        }
    }
    return p;
}

static int32_t sign_extend(int32_t v, int bits)
{
    int32_t sign = 1 << (bits - 1);
    v &= (1 << bits) - 1;
    return (v ^ sign) - sign;
}

/* Endpoint unquantisation: the format's integer form of eq. (6). The factor a
 * of eq. (6) (31/64 unsigned, 31/32 signed) is applied after interpolation,
 * in finish_unsigned/finish_signed below. */
static int32_t unquantize_unsigned(int32_t e, int bits)
{
    if (bits >= 15) return e;
    if (e == 0) return 0;
    if (e == (1 << bits) - 1) return 0xFFFF;
    return ((e << 16) + 0x8000) >> bits;
}

static int32_t unquantize_signed(int32_t e, int bits)
{
    if (bits >= 16) return e;
    int negative = e < 0;
    int32_t mag = negative ? -e : e;
    int32_t u;
    if (mag == 0) u = 0;
    else if (mag >= (1 << (bits - 1)) - 1) u = 0x7FFF;
    else u = ((mag << 15) + 0x4000) >> (bits - 1);
    return negative ? -u : u;
}

/* Weighted blend of the two unquantised endpoints (eq. 7), rounded to nearest
 * with floor division by 64. */
static int32_t interpolate(int32_t a, int32_t b, int weight)
{
    int64_t num = (int64_t)(64 - weight) * a + (int64_t)weight * b + 32;
    return (int32_t)floor((double)num / 64.0);
}

/* Scale by 31/64 and reinterpret as a positive half (eq. 8's bit cast). */
static uint16_t finish_unsigned(int32_t v)
{
    return (uint16_t)((v * 31) >> 6);
}

/* Scale the magnitude by 31/32 and set the half's sign bit for negatives. */
static uint16_t finish_signed(int32_t v)
{
    if (v < 0)
        return (uint16_t)((((-v) * 31) >> 5) | 0x8000);
    return (uint16_t)((v * 31) >> 5);
}

int bcfo_block_fields(const uint8_t block[16], int32_t fields[14])
{
    int mode_number;
    const mode_t *md = find_mode(block, &mode_number);
    memset(fields, 0, sizeof(int32_t) * 14);
    if (!md) return 0;
    int32_t f[F_COUNT];
    read_fields(block, md, f);
    int order[12] = {F_RW, F_GW, F_BW, F_RX, F_GX, F_BX, F_RY, F_GY, F_BY, F_RZ, F_GZ, F_BZ};
    for (int i = 0; i < 12; i++) fields[i] = f[order[i]];
    fields[12] = f[F_D];
    fields[13] = mode_number;
    return mode_number;
}

int bcfo_partition(int k, uint16_t *mask, int *anchor)
{
    if (k < 0 || k > 31) return -1;
    if (mask) *mask = PARTITION_MASK[k];
    if (anchor) *anchor = PARTITION_ANCHOR[k];
    return 0;
}

int bcfo_mode_bit_budget(int mode, int *header_bits, int *index_bits)
{
    if (mode < 1 || mode > 14) return -1;
    const mode_t *md = &MODES[mode - 1];
    int h = 0;
    for (int r = 0, n = run_count(md); r < n; r++)
        h += abs((int)md->runs[r].a - (int)md->runs[r].b) + 1;
    /* every texel stores an index of the mode's width except one anchor per
     * subset, which stores one bit fewer */
    int width = md->regions == 2 ? 3 : 4;
    int idx = 16 * width - md->regions;
    if (header_bits) *header_bits = h;
    if (index_bits) *index_bits = idx;
    return h + idx;
}

int bcfo_decode_block(const uint8_t block[16], int is_signed, uint16_t out[48])
{
    int mode_number;
    const mode_t *md = find_mode(block, &mode_number);
    memset(out, 0, sizeof(uint16_t) * 48);
    if (!md) return 0;                       /* reserved mode code: all zero */

    int32_t f[F_COUNT];
    int p = read_fields(block, md, f);

    /* endpoints e[j][c], j = w, x, y, z */
    int32_t e[4][3] = {
        {f[F_RW], f[F_GW], f[F_BW]},
        {f[F_RX], f[F_GX], f[F_BX]},
        {f[F_RY], f[F_GY], f[F_BY]},
        {f[F_RZ], f[F_GZ], f[F_BZ]},
    };
    int n_endpoints = 2 * md->regions;
    int eb = md->ep_bits;
    int mask = (1 << eb) - 1;

    if (is_signed)
        for (int c = 0; c < 3; c++) e[0][c] = sign_extend(e[0][c], eb);
    for (int j = 1; j < n_endpoints; j++)
        for (int c = 0; c < 3; c++) {
            if (md->transformed) {
                int32_t d = sign_extend(e[j][c], md->delta_bits[c]);
                e[j][c] = (e[0][c] + d) & mask;
                if (is_signed) e[j][c] = sign_extend(e[j][c], eb);
            } else if (is_signed) {
                e[j][c] = sign_extend(e[j][c], eb);
            }
        }

    int32_t unq[4][3];
    for (int j = 0; j < n_endpoints; j++)
        for (int c = 0; c < 3; c++)
            unq[j][c] = is_signed ? unquantize_signed(e[j][c], eb)
                                  : unquantize_unsigned(e[j][c], eb);

    int partition = md->regions == 2 ? f[F_D] : 0;
    int index_width = md->regions == 2 ? 3 : 4;
    int index[16];
    for (int t = 0; t < 16; t++) {
        int anchor = t == 0 || (md->regions == 2 && t == PARTITION_ANCHOR[partition]);
        int nb = index_width - anchor;
        index[t] = (int)block_bits(block, p, nb);
        p += nb;
    }

    for (int t = 0; t < 16; t++) {
        int subset = md->regions == 2 ? (PARTITION_MASK[partition] >> t) & 1 : 0;
        int weight = index_width == 3 ? WEIGHTS3[index[t]] : WEIGHTS4[index[t]];
        for (int c = 0; c < 3; c++) {
            int32_t v = interpolate(unq[2 * subset][c], unq[2 * subset + 1][c], weight);
            out[t * 3 + c] = is_signed ? finish_signed(v) : finish_unsigned(v);
        }
    }
    return mode_number;
}

void bcfo_decode_blocks(const uint8_t *blocks, size_t n, int is_signed, uint16_t *out)
{
    for (size_t i = 0; i < n; i++)
        bcfo_decode_block(blocks + 16 * i, is_signed, out + 48 * i);
}

/* ------------------------------------------------------------------------ */
/* Mip chains: level l is max(W>>l,1) x max(H>>l,1) texels stored as 4x4 blocks */

static uint32_t level_dim(uint32_t d, uint32_t level)
{
    uint32_t v = d >> level;
    return v ? v : 1;
}

static uint32_t blocks_across(uint32_t texels)
{
    return (texels + 3) / 4;
}

size_t bcfo_texture_bytes(uint32_t width, uint32_t height, uint32_t levels)
{
    size_t bytes = 0;
    for (uint32_t l = 0; l < levels; l++)
        bytes += (size_t)blocks_across(level_dim(width, l)) *
                 blocks_across(level_dim(height, l)) * 16;
    return bytes;
}

/* ------------------------------------------------------------------------ */
/* Filtering (Section "Hardware compliant filtering", eq. 9) */

static long wrap_index(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Texel (tx, ty) of level `level`, with wrap addressing, as three doubles. */
static void fetch_texel(const bcfo_texture *tex, int is_signed, uint32_t level,
                        long tx, long ty, double rgb[3])
{
    uint32_t w = level_dim(tex->width, level), h = level_dim(tex->height, level);
    tx = wrap_index(tx, w);
    ty = wrap_index(ty, h);
    size_t offset = bcfo_texture_bytes(tex->width, tex->height, level);
    size_t block = (size_t)(ty / 4) * blocks_across(w) + (size_t)(tx / 4);
    uint16_t texels[48];
    bcfo_decode_block(tex->blocks + offset + 16 * block, is_signed, texels);
    int t = (int)((ty % 4) * 4 + (tx % 4));
    for (int c = 0; c < 3; c++)
        rgb[c] = bcfo_half_to_double(texels[t * 3 + c]);
}

/* Bilinear interpolation T^k(u, v) on level k. Texel centres sit at
 * ((i + 1/2) / w, (j + 1/2) / h); addressing wraps in both directions. */
static void bilinear(const bcfo_texture *tex, int is_signed, uint32_t level,
                     double u, double v, double rgb[3])
{
    uint32_t w = level_dim(tex->width, level), h = level_dim(tex->height, level);
    double x = u * w - 0.5, y = v * h - 0.5;
    double x0 = floor(x), y0 = floor(y);
    double fx = x - x0, fy = y - y0;
    long ix = (long)x0, iy = (long)y0;
    double t00[3], t10[3], t01[3], t11[3];
    fetch_texel(tex, is_signed, level, ix, iy, t00);
    fetch_texel(tex, is_signed, level, ix + 1, iy, t10);
    fetch_texel(tex, is_signed, level, ix, iy + 1, t01);
    fetch_texel(tex, is_signed, level, ix + 1, iy + 1, t11);
    for (int c = 0; c < 3; c++)
        rgb[c] = (1 - fx) * (1 - fy) * t00[c] + fx * (1 - fy) * t10[c]
               + (1 - fx) * fy * t01[c] + fx * fy * t11[c];
}

/* T_i(u, v, s) = lambda T^{floor(s_i)+1}(u, v) + (1 - lambda) T^{floor(s_i)}(u, v)
 * with s_i = s + b_i clamped to [0, L-1] and the upper level clamped to L-1. */
static void trilinear(const bcfo_texture *tex, int is_signed, double u, double v,
                      double s, double rgb[3])
{
    if (!isfinite(u) || !isfinite(v) || isnan(s)) {
        rgb[0] = rgb[1] = rgb[2] = NAN;
        return;
    }
    /* Only u and v modulo one texture period matter under wrap addressing;
     * removing the integer part first is exact in binary64. */
    u -= floor(u);
    v -= floor(v);
    double s_i = s + tex->lod_bias;
    double top = (double)(tex->levels - 1);
    if (s_i < 0) s_i = 0;
    if (s_i > top) s_i = top;
    uint32_t l0 = (uint32_t)floor(s_i);
    uint32_t l1 = l0 + 1 < tex->levels ? l0 + 1 : tex->levels - 1;
    double lambda = s_i - l0;
    double a[3], b[3];
    bilinear(tex, is_signed, l0, u, v, a);
    bilinear(tex, is_signed, l1, u, v, b);
    for (int c = 0; c < 3; c++)
        rgb[c] = lambda * b[c] + (1 - lambda) * a[c];
}

static void sample_one(const bcfo_material *m, const float *q, double *feat)
{
    for (uint32_t i = 0; i < m->n_textures; i++)
        trilinear(&m->textures[i], m->is_signed, q[0], q[1], q[2], feat + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Decoder MLP f_eta: ReLU hidden layers, linear output layer */

static void mlp_one(const bcfo_material *m, const double *z_in, double *out)
{
    double buf_a[1024], buf_b[1024];
    const float *p = m->params;
    const double *z = z_in;
    double *y = buf_a;
    for (uint32_t l = 0; l < m->n_layers; l++) {
        uint32_t n_in = m->dims[l], n_out = m->dims[l + 1];
        const float *W = p, *b = p + (size_t)n_in * n_out;
        int last = l + 1 == m->n_layers;
        double *dst = last ? out : y;
        for (uint32_t j = 0; j < n_out; j++) {
            double acc = b[j];
            for (uint32_t i = 0; i < n_in; i++)
                acc += (double)W[(size_t)j * n_in + i] * z[i];
            dst[j] = (!last && acc < 0) ? 0.0 : acc;
        }
        p += (size_t)n_in * n_out + n_out;
        z = dst;
        y = (y == buf_a) ? buf_b : buf_a;
    }
}

void bcfo_mlp(const bcfo_material *m, const double *z, size_t n, double *out)
{
    uint32_t n_in = m->dims[0], n_out = m->dims[m->n_layers];
    for (size_t q = 0; q < n; q++)
        mlp_one(m, z + q * n_in, out + q * n_out);
}

/* ------------------------------------------------------------------------ */
/* Whole decode, split over threads by contiguous query ranges */

typedef struct {
    const bcfo_material *m;
    const float *queries;
    size_t begin, end;
    double *out;
    int features_only;
} job_t;

static void *run_job(void *arg)
{
    job_t *job = (job_t *)arg;
    const bcfo_material *m = job->m;
    uint32_t n_feat = 3 * m->n_textures;
    uint32_t n_out = job->features_only ? n_feat : m->dims[m->n_layers];
    double feat[3 * 64];
    for (size_t q = job->begin; q < job->end; q++) {
        double *dst = job->out + q * n_out;
        sample_one(m, job->queries + 3 * q, job->features_only ? dst : feat);
        if (!job->features_only)
            mlp_one(m, feat, dst);
    }
    return NULL;
}

static void run_parallel(const bcfo_material *m, const float *queries, size_t n,
                         double *out, int n_threads, int features_only)
{
    if (n_threads < 1) n_threads = 1;
    if ((size_t)n_threads > n) n_threads = n ? (int)n : 1;
    job_t *jobs = calloc((size_t)n_threads, sizeof(job_t));
    pthread_t *threads = calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; t++) {
        jobs[t].m = m;
        jobs[t].queries = queries;
        jobs[t].begin = n * (size_t)t / n_threads;
        jobs[t].end = n * (size_t)(t + 1) / n_threads;
        jobs[t].out = out;
        jobs[t].features_only = features_only;
    }
    for (int t = 1; t < n_threads; t++)
        pthread_create(&threads[t], NULL, run_job, &jobs[t]);
    run_job(&jobs[0]);
    for (int t = 1; t < n_threads; t++)
        pthread_join(threads[t], NULL);
    free(jobs);
    free(threads);
}

void bcfo_sample(const bcfo_material *m, const float *queries, size_t n,
                 double *feats, int n_threads)
{
    run_parallel(m, queries, n, feats, n_threads, 1);
}

void bcfo_decode(const bcfo_material *m, const float *queries, size_t n,
                 double *out, int n_threads)
{
    run_parallel(m, queries, n, out, n_threads, 0);
}
