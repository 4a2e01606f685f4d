// Trilinear filtering of the feature pyramids from the texel scratch
// (eq. 9 at s_i = s + b_i of eq. 10), for the decode kernels.
//
// Texel scratch: level l of pyramid t is max(h>>l,1) rows of pitch w_l + 2
// texels of 8 bytes (r | g << 16, b as half bit patterns). Column w_l repeats
// texel 0 of its row, so the two horizontal taps of a bilinear footprint are
// one 16-byte load, also across the wrap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace bcf {

__host__ __device__ inline uint32_t row_pitch(uint32_t w) { return w + 2u; }

// Per pyramid slot and level, as the kernels read it from LDS:
//   x = float(w_l), y = float(h_l), z = (w_l - 1) | (h_l - 1) << 16, w = first texel
struct LevelLut {
    uint4 e[kMaxTextures][kMaxLevels];
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    // raw buffer: 32-bit byte offsets; loads past `bytes` return 0, stores are dropped
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float half_lo(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu));
}

__device__ __forceinline__ float half_hi(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}

struct LevelSel {
    uint32_t l0, l1;
    float lam;
};

__device__ __forceinline__ LevelSel select_levels(float s, float bias, uint32_t levels)
{
    // s_i = s + b_i clamped to [0, L-1]; fmaxf maps NaN to 0
    const float si = fminf(fmaxf(s + bias, 0.0f), (float)(levels - 1));
    const float lf = floorf(si);
    LevelSel r;
    r.l0 = (uint32_t)lf;
    r.l1 = min(r.l0 + 1, levels - 1);
    r.lam = si - lf;
    return r;
}

// One level's bilinear footprint: byte offsets of the texel pairs
// (x0, y0)+(x0+1, y0) and (x0, y1)+(x0+1, y1), and the four weights scaled
// by the level's trilinear weight lw.
struct Footprint {
    uint32_t o0, o1;
    float w00, w10, w01, w11;
};

// The integer texel coordinates of a level's bilinear footprint: columns x0
// and x0 + 1 (x0 + 1 = w is the wrap column, a copy of column 0), rows y0 and
// y1, and the fractional parts. Shared by the filters and the batch's marking
// of the blocks a set of queries touches, so both take the same taps.
struct TapCoords {
    uint32_t x0, y0, y1, wm;
    float fx, fy;
};

__device__ __forceinline__ TapCoords tap_coords(uint4 e, float uf, float vf)
{
#pragma clang fp contract(off)
    // copy the fields to plain integers before reinterpreting them
    const uint32_t ew = e.x, eh = e.y, masks = e.z;
    const float x = fmaf(uf, __builtin_bit_cast(float, ew), -0.5f);
    const float y = fmaf(vf, __builtin_bit_cast(float, eh), -0.5f);
    TapCoords t;
    t.fx = __builtin_amdgcn_fractf(x);
    t.fy = __builtin_amdgcn_fractf(y);
    t.wm = masks & 0xFFFFu;
    const uint32_t hm = masks >> 16;
    t.x0 = (uint32_t)(int)floorf(x) & t.wm;                     // -1 wraps to w-1
    t.y0 = (uint32_t)(int)floorf(y) & hm;
    t.y1 = (t.y0 + 1u) & hm;
    return t;
}

// UNIT: bytes per texel slot of the scratch (8; 24 for a packed one, whose
// LUT offsets count 24-byte positions)
template <uint32_t UNIT = 8>
__device__ __forceinline__ Footprint footprint(uint4 e, float uf, float vf, float lw)
{
    // every product and sum below is rounded as written, whichever kernel
    // this is inlined into, so all decode kernels filter bit-identically
#pragma clang fp contract(off)
    const uint32_t first = e.w;
    const TapCoords t = tap_coords(e, uf, vf);
    const float fx = t.fx, fy = t.fy;
    const uint32_t x0 = t.x0, y0 = t.y0, y1 = t.y1;
    const uint32_t lw2 = __builtin_popcount(t.wm);              // log2 w
    // row y starts at y * (w + 2) = (y << log2 w) + 2 y
    Footprint f;
    f.o0 = ((y0 << lw2) + 2u * y0 + x0 + first) * UNIT;
    f.o1 = ((y1 << lw2) + 2u * y1 + x0 + first) * UNIT;
    const float wx1 = fx * lw, wx0 = fmaf(-fx, lw, lw);
    f.w01 = wx0 * fy;
    f.w11 = wx1 * fy;
    f.w00 = fmaf(-wx0, fy, wx0);
    f.w10 = fmaf(-wx1, fy, wx1);
    return f;
}

typedef uint32_t texel_pair __attribute__((ext_vector_type(4)));   // two 8-byte texels

// acc[0..2] += the footprint's weighted texels from its two fetched rows
__device__ __forceinline__ void blend(const Footprint &f, texel_pair r0, texel_pair r1, float *acc)
{
    acc[0] = fmaf(f.w00, half_lo(r0[0]), acc[0]);
    acc[0] = fmaf(f.w10, half_lo(r0[2]), acc[0]);
    acc[0] = fmaf(f.w01, half_lo(r1[0]), acc[0]);
    acc[0] = fmaf(f.w11, half_lo(r1[2]), acc[0]);
    acc[1] = fmaf(f.w00, half_hi(r0[0]), acc[1]);
    acc[1] = fmaf(f.w10, half_hi(r0[2]), acc[1]);
    acc[1] = fmaf(f.w01, half_hi(r1[0]), acc[1]);
    acc[1] = fmaf(f.w11, half_hi(r1[2]), acc[1]);
    acc[2] = fmaf(f.w00, half_lo(r0[1]), acc[2]);
    acc[2] = fmaf(f.w10, half_lo(r0[3]), acc[2]);
    acc[2] = fmaf(f.w01, half_lo(r1[1]), acc[2]);
    acc[2] = fmaf(f.w11, half_lo(r1[3]), acc[2]);
}

// acc[0..2] += the footprint's weighted texels, the level starting `shift`
// bytes after the footprint's own base
__device__ __forceinline__ void gather(__amdgpu_buffer_rsrc_t rs, const Footprint &f, uint32_t shift,
                                      float *acc)
{
    const texel_pair r0 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(f.o0 + shift), 0, 0);
    const texel_pair r1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(f.o1 + shift), 0, 0);
    blend(f, r0, r1, acc);
}

// A query's trilinear footprint for pyramids of one shared geometry, with its
// 16 texel-pair loads issued (4 slots x 2 levels x 2 rows), so the frame
// kernel can fetch the next work item before storing the current one.
struct PendingTaps {
    Footprint f0, f1;
    texel_pair r[kMaxTextures][2][2];
};

__device__ __forceinline__ void fetch4_shared(__amdgpu_buffer_rsrc_t rs, const LevelLut &lut,
                                              const float *levels_bias, uint32_t stride, float u, float v,
                                              float s, PendingTaps &p)
{
    const float uf = u - floorf(u), vf = v - floorf(v);       // wrap addressing
    const LevelSel ls = select_levels(s, levels_bias[1], __builtin_bit_cast(uint32_t, levels_bias[0]));
    p.f0 = footprint(lut.e[0][ls.l0], uf, vf, 1.0f - ls.lam);
    p.f1 = footprint(lut.e[0][ls.l1], uf, vf, ls.lam);
#pragma unroll
    for (int t = 0; t < kMaxTextures; ++t) {
        const uint32_t sh = (uint32_t)t * stride;
        p.r[t][0][0] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(p.f0.o0 + sh), 0, 0);
        p.r[t][0][1] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(p.f0.o1 + sh), 0, 0);
        p.r[t][1][0] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(p.f1.o0 + sh), 0, 0);
        p.r[t][1][1] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(p.f1.o1 + sh), 0, 0);
    }
}

// A query's trilinear footprint on a packed scratch (MaterialDesc::interleaved):
// position x of a level holds the four pyramids' (r, g, b) halves, 24 bytes,
// so a footprint row of all four is the 48 bytes of positions x0 and x0 + 1,
// three 16-byte loads (four 8-byte texels per position would take four). q[level][row][k] = bytes 16k .. 16k + 15 of the row's span.
struct PendingPacked {
    Footprint f0, f1;
    texel_pair q[2][2][3];
};

__device__ __forceinline__ void fetch4_packed(__amdgpu_buffer_rsrc_t rs, const LevelLut &lut,
                                              const float *levels_bias, float u, float v, float s,
                                              PendingPacked &p)
{
    const float uf = u - floorf(u), vf = v - floorf(v);       // wrap addressing
    const LevelSel ls = select_levels(s, levels_bias[1], __builtin_bit_cast(uint32_t, levels_bias[0]));
    p.f0 = footprint<24>(lut.e[0][ls.l0], uf, vf, 1.0f - ls.lam);
    p.f1 = footprint<24>(lut.e[0][ls.l1], uf, vf, ls.lam);
    const uint32_t off[2][2] = {{p.f0.o0, p.f0.o1}, {p.f1.o0, p.f1.o1}};
#pragma unroll
    for (int lv = 0; lv < 2; ++lv)
#pragma unroll
        for (int row = 0; row < 2; ++row)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                p.q[lv][row][k] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off[lv][row] + 16u * k), 0, 0);
}

// Half h (0..23) of a packed footprint row: position h / 12, pyramid
// (h % 12) / 3, channel h % 3.
__device__ __forceinline__ float packed_half(const texel_pair (&q)[3], int h)
{
    const uint32_t d = q[h >> 3][(h >> 1) & 3];
    return (h & 1) ? half_hi(d) : half_lo(d);
}

// filter_pending for packed taps: the same sums in the same order (per
// pyramid and channel: level l0's four taps, then level l1's).
__device__ __forceinline__ void filter_pending_packed(const PendingPacked &p, float z[12])
{
#pragma unroll
    for (int i = 0; i < 12; ++i) z[i] = 0.0f;
#pragma unroll
    for (int lv = 0; lv < 2; ++lv) {
        const Footprint &f = lv ? p.f1 : p.f0;
#pragma unroll
        for (int i = 0; i < 12; ++i) {           // i = 3 t + c: halves i (x0) and 12 + i (x0 + 1)
            z[i] = fmaf(f.w00, packed_half(p.q[lv][0], i), z[i]);
            z[i] = fmaf(f.w10, packed_half(p.q[lv][0], 12 + i), z[i]);
            z[i] = fmaf(f.w01, packed_half(p.q[lv][1], i), z[i]);
            z[i] = fmaf(f.w11, packed_half(p.q[lv][1], 12 + i), z[i]);
        }
    }
}

// the sums of filter4<true> from fetched taps
__device__ __forceinline__ void filter_pending(const PendingTaps &p, float z[12])
{
#pragma unroll
    for (int i = 0; i < 12; ++i) z[i] = 0.0f;
#pragma unroll
    for (int t = 0; t < kMaxTextures; ++t) {
        blend(p.f0, p.r[t][0][0], p.r[t][0][1], z + 3 * t);
        blend(p.f1, p.r[t][1][0], p.r[t][1][1], z + 3 * t);
    }
}

// Scratch layouts of a single material's decode: each pyramid's own levels
// (kLayoutSplit), the same with one shared geometry, slot t t * stride bytes
// after slot 0 (kLayoutShared), or four pyramids of one geometry packed per
// position (kLayoutPacked).
constexpr int kLayoutSplit = 0, kLayoutShared = 1, kLayoutPacked = 2;

// z[3t + c] = T_t(u, v, s) channel c for the four pyramid slots (slots past
// the material's pyramids repeat slot 0; their MLP weights are zero).
// kLayoutShared / kLayoutPacked: every slot has the same w, h, levels and
// bias, so one footprint serves all four.
template <int LAYOUT>
__device__ __forceinline__ void filter4(__amdgpu_buffer_rsrc_t rs, const LevelLut &lut,
                                        const float *levels_bias, uint32_t stride, float u, float v,
                                        float s, float z[12])
{
    if (LAYOUT == kLayoutPacked) {
        PendingPacked p;
        fetch4_packed(rs, lut, levels_bias, u, v, s, p);
        filter_pending_packed(p, z);
        return;
    }
    const float uf = u - floorf(u), vf = v - floorf(v);       // wrap addressing
#pragma unroll
    for (int i = 0; i < 12; ++i) z[i] = 0.0f;
    if (LAYOUT == kLayoutShared) {
        const LevelSel ls = select_levels(s, levels_bias[1], __builtin_bit_cast(uint32_t, levels_bias[0]));
        const Footprint f0 = footprint(lut.e[0][ls.l0], uf, vf, 1.0f - ls.lam);
        const Footprint f1 = footprint(lut.e[0][ls.l1], uf, vf, ls.lam);
#pragma unroll
        for (int t = 0; t < kMaxTextures; ++t) {
            gather(rs, f0, (uint32_t)t * stride, z + 3 * t);
            gather(rs, f1, (uint32_t)t * stride, z + 3 * t);
        }
    } else {
#pragma unroll
        for (int t = 0; t < kMaxTextures; ++t) {
            const LevelSel ls = select_levels(s, levels_bias[2 * t + 1],
                                              __builtin_bit_cast(uint32_t, levels_bias[2 * t]));
            const Footprint f0 = footprint(lut.e[t][ls.l0], uf, vf, 1.0f - ls.lam);
            const Footprint f1 = footprint(lut.e[t][ls.l1], uf, vf, ls.lam);
            gather(rs, f0, 0, z + 3 * t);
            gather(rs, f1, 0, z + 3 * t);
        }
    }
}

}  // namespace bcf
