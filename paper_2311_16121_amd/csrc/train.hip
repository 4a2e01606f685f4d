// Training-time decode for gfx950: forward and backward through the simulated
// BC6H decompression of Section 4.2 (eqs. 6-8), the trilinear filter (eqs. 9
// and 10) and the ReLU MLP (eq. 3).
//
//   k_train_texels    block parameters -> texel images (r, g, b, 0) per level
//   k_train_forward_mfma  queries -> G(u, v, s), one lane per query, the MLP
//                     on the matrix cores
//   k_train_bin_*     the backward's samples sorted by position (counting
//                     sort over a grid of cells on the wrapped (u, v))
//   k_train_backward  queries, dL/dG -> dL/d features per sample and dL/d MLP
//                     parameters (per-wave sums on the matrix cores)
//   k_train_scatter   dL/d features -> dL/d texel, one workgroup per cell:
//                     fixed-point sums in LDS windows over the cell's
//                     footprint, then one float atomic per touched texel channel
//   k_train_blocks    dL/d texel -> dL/d endpoints, dL/d indices (one lane
//                     per texel, sums over a block's 16 lanes by shuffles)
//
// A texel of subset sigma blends the endpoint pair (e_{2 sigma}, e_{2 sigma+1})
// with index x. Continuous mode: y = a ((2^16 e_A + 2^15)/2^6 + x (2^16 (e_B -
// e_A))/2^6), w = eq. (8) of y. Straight-through mode: w is the format's exact
// decode of the rounded endpoints and index (i = rint(7 x)); the derivatives are
// those of the continuous chain at the rounded point (x = w_i / 64), with the
// rounding taken as the identity and eq. (8)'s slope at the decoded bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bc6h_device.hpp"
#include "frame_kernels.hpp"
#include "train.hpp"

namespace bcf {
namespace {

constexpr float kA = 31.0f / 64.0f;      // a of eq. (6) for the unsigned format
constexpr int kTrainThreads = 256;

__global__ void __launch_bounds__(256) k_train_zero(float *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// one texel channel

struct TexelChan {
    float w;              // texel value
    float slope;          // dw/dy of eq. (8)
    float dy_da, dy_db;   // dy/d e_A, dy/d e_B
    float dy_dx;          // dy/d x
};

// h(y) = max(floor((y - 1) / 1024) - 1, 0) of eq. (8) for integer y >= 0
__device__ __forceinline__ int h_of_bits(uint32_t y)
{
    const int k = y ? (int)((y - 1u) >> 10) - 1 : 0;
    return k > 0 ? k : 0;
}

template <bool STE>
__device__ __forceinline__ TexelChan texel_chan(float ea, float eb, float x)
{
    TexelChan r;
    if (!STE) {
        // (2^16 e + 2^15) / 2^6 = 1024 e + 512, exact in binary32 for e in [0, 64)
        const float abar = fmaf(1024.0f, ea, 512.0f);
        const float bbar = fmaf(1024.0f, eb, 512.0f);
        const float y = kA * fmaf(x, bbar - abar, abar);
        const float h = fmaxf(floorf((y - 1.0f) * (1.0f / 1024.0f)) - 1.0f, 0.0f);
        r.w = ldexpf(y * (1.0f / 1024.0f) - h, (int)h - 14);
        r.slope = ldexpf(1.0f, (int)h - 24);
        r.dy_da = kA * 1024.0f * (1.0f - x);
        r.dy_db = kA * 1024.0f * x;
        r.dy_dx = kA * (bbar - abar);
    } else {
        // fmaxf before fminf maps NaN to 0
        const float qa = fminf(fmaxf(rintf(ea), 0.0f), 63.0f);
        const float qb = fminf(fmaxf(rintf(eb), 0.0f), 63.0f);
        const uint32_t i = (uint32_t)fminf(fmaxf(rintf(7.0f * x), 0.0f), 7.0f);
        const int32_t wt = (int32_t)((i * 585u + 32u) >> 6);       // round(64 i / 7)
        const int32_t A = unquantize<false>((int32_t)qa, 6);
        const int32_t B = unquantize<false>((int32_t)qb, 6);
        const int32_t v = ((64 - wt) * A + wt * B + 32) >> 6;
        const uint32_t y = ((uint32_t)v * 31u) >> 6;
        r.w = (float)__builtin_bit_cast(_Float16, (uint16_t)y);
        r.slope = ldexpf(1.0f, h_of_bits(y) - 24);
        const float xs = (float)wt * (1.0f / 64.0f);
        r.dy_da = kA * 1024.0f * (1.0f - xs);
        r.dy_db = kA * 1024.0f * xs;
        r.dy_dx = kA * 1024.0f * (qb - qa);
    }
    return r;
}

// Where texel t of joint block gb lives: pyramid, block within it, level and
// position; false for the texels a level below 4x4 does not have.
struct TexelSite {
    uint32_t ti, b, x, y, tex;      // tex: texel index in the images
    uint32_t wl;                    // the level's width
    bool valid;
};

__device__ __forceinline__ TexelSite texel_site(const TrainDesc &d, uint32_t gb, uint32_t t)
{
    TexelSite s;
    uint32_t ti = 0;
    while (ti + 1 < d.n_tex && gb >= d.blk_base[ti + 1]) ++ti;
    const TrainTexDesc &tx = d.tex[ti];
    const uint32_t b = gb - d.blk_base[ti];
    uint32_t l = 0;
    while (l + 1 < tx.levels && b >= tx.blk_off[l + 1]) ++l;
    const uint32_t wl = max(tx.w >> l, 1u), hl = max(tx.h >> l, 1u);
    const uint32_t bxn = (wl + 3u) >> 2;          // a power of two, as the level width is
    const uint32_t lb = b - tx.blk_off[l];
    s.ti = ti;
    s.b = b;
    s.x = (lb & (bxn - 1u)) * 4u + (t & 3u);
    s.y = (lb >> __builtin_ctz(bxn)) * 4u + (t >> 2);
    s.valid = s.x < wl && s.y < hl;
    s.tex = tx.tex_off[l] + s.y * wl + s.x;
    s.wl = wl;
    return s;
}

__device__ __forceinline__ uint32_t subset_of(const TrainTexDesc &tx, uint32_t b, uint32_t t)
{
    // partition ids are taken modulo 32
    return (kTable[kModes * kModeWords + (tx.partitions[b] & 31u)] >> t) & 1u;
}

// One lane per block row: its four texels (a level narrower than 4 texels
// keeps the left ones), the block's endpoints and partition read once.
template <bool STE>
__global__ void __launch_bounds__(kTrainThreads) k_train_texels(TrainDesc d)
{
    const uint32_t total = d.blk_base[d.n_tex] * 4u;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
        const uint32_t r = g & 3u;
        const TexelSite s = texel_site(d, g >> 2, 4u * r);
        if (!s.valid) continue;
        const TrainTexDesc &tx = d.tex[s.ti];
        // partition ids are taken modulo 32
        const uint32_t pmask = kTable[kModes * kModeWords + (tx.partitions[s.b] & 31u)];
        float e[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) e[k] = tx.endpoints[12u * s.b + k];
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            if (s.x + i >= s.wl) break;
            const uint32_t t = 4u * r + i, sub = (pmask >> t) & 1u;
            const float x = tx.indices[16u * s.b + t];
            float w[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) w[c] = texel_chan<STE>(sub ? e[6 + c] : e[c], sub ? e[9 + c] : e[3 + c], x).w;
            d.texels[s.tex + i] = make_float4(w[0], w[1], w[2], 0.0f);
        }
    }
}

// Sum over the 16 lanes of a DPP row (a block's texels), in every lane of the
// row: lanes paired by XOR 1, then 2, then the row's two quads of each half,
// then its two halves -- the order of a shuffle butterfly over XOR 1, 2, 4, 8,
// with DPP moves instead of LDS permutes.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float row16_sum(float v)
{
    v += dpp_move<0xB1>(v);       // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);       // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);      // row_half_mirror: lane i of a half row takes lane 7 - i
    v += dpp_move<0x140>(v);      // row_mirror: lane i takes lane 15 - i
    return v;
}

template <bool STE>
__global__ void __launch_bounds__(kTrainThreads) k_train_blocks(TrainDesc d)
{
    // every 16-lane group is one block: total is a multiple of 16, so a group's
    // lanes enter and leave the loop together
    const uint32_t total = d.blk_base[d.n_tex] * 16u;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
        const uint32_t t = g & 15u;
        const TexelSite s = texel_site(d, g >> 4, t);
        const TrainTexDesc &tx = d.tex[s.ti];
        const uint32_t sub = subset_of(tx, s.b, t);
        const float *e = tx.endpoints + 12u * s.b;
        float gx = 0.0f;
        float ge[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};   // this texel's pair A, B
        if (s.valid) {
            const float4 gt = d.g_texels[s.tex];
            const float gc[3] = {gt.x, gt.y, gt.z};
            const float x = tx.indices[16u * s.b + t];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const TexelChan r = texel_chan<STE>(e[6u * sub + c], e[6u * sub + 3u + c], x);
                const float gy = gc[c] * r.slope;
                gx = fmaf(gy, r.dy_dx, gx);
                ge[0][c] = gy * r.dy_da;
                ge[1][c] = gy * r.dy_db;
            }
        }
        tx.g_indices[16u * s.b + t] = gx;
        // sum over the block's texels, per subset
        float sum[4][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sum[0][c] = sub ? 0.0f : ge[0][c];
            sum[1][c] = sub ? 0.0f : ge[1][c];
            sum[2][c] = sub ? ge[0][c] : 0.0f;
            sum[3][c] = sub ? ge[1][c] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sum[j][c] = row16_sum(sum[j][c]);
        if (t < 12) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) v = (3 * j + c == (int)t) ? sum[j][c] : v;
            tx.g_endpoints[12u * s.b + t] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// queries

// Per pyramid and level, for the query kernels' LDS: x = level width,
// y = level height, z = first texel of the level in the images. A level picked
// per query indexes it; indexing the descriptor's arrays instead makes the
// compiler hold every level's values in registers across the query loop.
typedef uint4 TrainLevelLut[kMaxTextures][kMaxLevels];

// Every thread of the workgroup takes part; the caller synchronises.
__device__ __forceinline__ void load_level_lut(const TrainDesc &d, TrainLevelLut &lut)
{
    for (uint32_t e = threadIdx.x; e < (uint32_t)(kMaxTextures * kMaxLevels); e += blockDim.x) {
        const uint32_t ti = e / kMaxLevels, l = e % kMaxLevels;
        const TrainTexDesc &tx = d.tex[ti < d.n_tex ? ti : 0u];
        lut[ti][l] = l < tx.levels ? make_uint4(max(tx.w >> l, 1u), max(tx.h >> l, 1u), tx.tex_off[l], 0u)
                                   : make_uint4(1u, 1u, 0u, 0u);
    }
}

// The four bilinear taps of wrapped (uf, vf) on one level (e = its LUT entry:
// width, height, first texel) and their weights times the level weight lw:
// columns xa, xb = xa + 1 and rows ya, yb = ya + 1 (wrapped); w[] in the order
// (ya, xa), (ya, xb), (yb, xa), (yb, xb).
struct LevelTaps {
    uint32_t xa, xb, ya, yb;
    float w[4];
};

__device__ __forceinline__ LevelTaps level_taps(uint4 e, float uf, float vf, float lw)
{
    LevelTaps r;
    const uint32_t wl = e.x, hl = e.y;
    const float x = fmaf(uf, (float)wl, -0.5f), y = fmaf(vf, (float)hl, -0.5f);
    const float x0 = floorf(x), y0 = floorf(y);
    const float fx = x - x0, fy = y - y0;
    r.xa = (uint32_t)(int)x0 & (wl - 1u);
    r.xb = (r.xa + 1u) & (wl - 1u);
    r.ya = (uint32_t)(int)y0 & (hl - 1u);
    r.yb = (r.ya + 1u) & (hl - 1u);
    r.w[0] = lw * (1.0f - fx) * (1.0f - fy);
    r.w[1] = lw * fx * (1.0f - fy);
    r.w[2] = lw * (1.0f - fx) * fy;
    r.w[3] = lw * fx * fy;
    return r;
}

// The 32 taps of a query (4 pyramids x 2 levels x 4 texels): texel index and
// weight (bilinear times trilinear); pyramids past n_tex get weight 0.
__device__ __forceinline__ void taps(const TrainDesc &d, const TrainLevelLut &lut, float u, float v, float s,
                                     uint32_t idx[32], float wt[32])
{
    const float uf = u - floorf(u), vf = v - floorf(v);          // wrap addressing
#pragma unroll
    for (int ti = 0; ti < kMaxTextures; ++ti) {
        const TrainTexDesc &tx = d.tex[ti < (int)d.n_tex ? ti : 0];
        const uint32_t slot = ti < (int)d.n_tex ? (uint32_t)ti : 0u;
        const float si = fminf(fmaxf(s + tx.bias, 0.0f), (float)(tx.levels - 1));   // NaN -> 0
        const uint32_t l0 = (uint32_t)floorf(si);
        const uint32_t l1 = min(l0 + 1u, tx.levels - 1u);
        const float lam = si - (float)l0;
        const float on = ti < (int)d.n_tex ? 1.0f : 0.0f;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const uint32_t l = k ? l1 : l0;
            const float lw = on * (k ? lam : 1.0f - lam);
            const uint4 e = lut[slot][l];
            const LevelTaps lt = level_taps(e, uf, vf, lw);
            const uint32_t wl = e.x, base = e.z;
            const int o = 8 * ti + 4 * k;
            idx[o + 0] = base + lt.ya * wl + lt.xa;
            idx[o + 1] = base + lt.ya * wl + lt.xb;
            idx[o + 2] = base + lt.yb * wl + lt.xa;
            idx[o + 3] = base + lt.yb * wl + lt.xb;
#pragma unroll
            for (int i = 0; i < 4; ++i) wt[o + i] = lt.w[i];
        }
    }
}

__device__ __forceinline__ void features(const TrainDesc &d, const TrainLevelLut &lut, float u, float v, float s,
                                         float z[12])
{
    uint32_t idx[32];
    float wt[32];
    taps(d, lut, u, v, s, idx, wt);
#pragma unroll
    for (int i = 0; i < 12; ++i) z[i] = 0.0f;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const float4 tv = d.texels[idx[k]];
        const int t = k / 8;
        z[3 * t + 0] = fmaf(wt[k], tv.x, z[3 * t + 0]);
        z[3 * t + 1] = fmaf(wt[k], tv.y, z[3 * t + 1]);
        z[3 * t + 2] = fmaf(wt[k], tv.z, z[3 * t + 2]);
    }
}

// The MLP's parameters in LDS, one padded row per neuron: its weights, its
// bias, zeros (layer 0's inputs padded to 12, the output layer to kMaxOut
// rows). The backward's matrix-core products read a weight (or, for the
// deltas, its transpose) per lane from these rows.
template <int H, int NH>
struct __align__(16) MlpLds {
    float w0[H][16];                          // inputs 0..11, bias at 12
    float wh[NH > 1 ? NH - 1 : 1][H][H + 4];  // inputs 0..H-1, bias at H
    float wl[kMaxOut][H + 4];
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
// Every thread of the workgroup takes part; synchronises the workgroup.
template <int H, int NH>
__device__ __forceinline__ void load_mlp(const TrainDesc &d, MlpLds<H, NH> &m)
{
    const uint32_t n0 = d.dims[0], c = d.dims[NH + 1];
    const float *P = d.params;
    for (uint32_t e = threadIdx.x; e < (uint32_t)(H * 16); e += blockDim.x) {
        const uint32_t j = e / 16u, i = e % 16u;
        m.w0[j][i] = i < n0 ? P[d.w_off[0] + j * n0 + i] : (i == 12 ? P[d.b_off[0] + j] : 0.0f);
    }
    for (uint32_t e = threadIdx.x; e < (uint32_t)((NH - 1) * H * (H + 4)); e += blockDim.x) {
        const uint32_t l = e / (H * (H + 4)), r = e % (H * (H + 4)), j = r / (H + 4), i = r % (H + 4);
        m.wh[l][j][i] = i < H ? P[d.w_off[l + 1] + j * H + i] : (i == H ? P[d.b_off[l + 1] + j] : 0.0f);
    }
    for (uint32_t e = threadIdx.x; e < (uint32_t)(kMaxOut * (H + 4)); e += blockDim.x) {
        const uint32_t j = e / (H + 4), i = e % (H + 4);
        m.wl[j][i] = j >= c ? 0.0f : i < H ? P[d.w_off[NH] + j * H + i] : (i == H ? P[d.b_off[NH] + j] : 0.0f);
    }
    __syncthreads();
}

// The forward with the MLP on the matrix cores (fp32 16x16x4 MFMAs, the
// decode kernels' operand layout, prepared from the parameters per call): a
// wave's 64 queries' features pass through LDS into the MFMA B layout, the
// outputs come back through LDS to each query's lane.
template <int H, int NH>
__global__ void __launch_bounds__(kTrainThreads) k_train_forward_mfma(TrainDesc d, const float *queries, uint32_t n,
                                                                      float *out)
{
    constexpr int kWaves = kTrainThreads / 64;
    __shared__ TrainLevelLut lut;
    __shared__ float4_t stage[kWaves][64 * kMaxOut / 4];     // features, then output rows
    load_level_lut(d, lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = d.dims[NH + 1];
    MfmaMlp<MLP_MFMA_F32, H, NH> mlp;
    mlp.load(d.ops_ws, d.ops, lane);
    float *st = reinterpret_cast<float *>(&stage[wv][0]);
    float4_t (*feats)[4] = reinterpret_cast<float4_t (*)[4]>(&stage[wv][0]);
    const uint32_t n_chunks = (n + 63u) / 64u;
    for (uint32_t ch = blockIdx.x * kWaves + wv; ch < n_chunks; ch += gridDim.x * kWaves) {
        const uint32_t q = ch * 64u + lane;
        const bool live = q < n;
        float z[12];
        features(d, lut, live ? queries[3u * q] : 0.0f, live ? queries[3u * q + 1u] : 0.0f,
                 live ? queries[3u * q + 2u] : 0.0f, z);
        mlp_stage<MLP_MFMA_F32, H, NH, kMaxOut>(z, d.ops_ws, d.ops, mlp, feats, st, c, lane);
        if (live)
            for (uint32_t j = 0; j < c; ++j) out[(size_t)q * c + j] = st[lane * c + j];
        wave_lds_sync();                              // the stage is rewritten by the next chunk
    }
}

// A layer's parameter gradients, dL/dW[j][i] = sum over queries of
// delta[q][j] * a[q][i], summed per wave on the matrix cores: 16 x 16 tiles
// (rows j = 16 m + .., columns i = 16 n + ..) of fp32 16x16x4 MFMAs, K running
// over the wave's 64 queries; at step s lane L supplies dl[4 s + L / 16][16 m
// + L % 16] and a[4 s + L / 16][16 n + L % 16], and tile register k of lane L
// holds row 4 (L / 16) + k, column L % 16. The bias gradients (sum over
// queries of delta[q][j]) are the per-lane sums of the same dl reads, added
// across the four lane groups when flushed.
template <int MT, int NT>
struct LayerGrad {
    f32x4 w[MT][NT];
    float b[MT];
};

template <int MT, int NT>
__device__ __forceinline__ void grad_zero(LayerGrad<MT, NT> &g)
{
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        g.b[m] = 0.0f;
#pragma unroll
        for (int n = 0; n < NT; ++n) g.w[m][n] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    }
}

template <int MT, int NT>
__device__ __forceinline__ void accumulate(LayerGrad<MT, NT> &g, const float (*a)[kTrainMaxHidden + 1],
                                           const float (*dl)[kTrainMaxHidden], uint32_t lane)
{
    static_assert(16 * MT <= kTrainMaxHidden && 16 * NT <= kTrainMaxHidden, "tiles inside the LDS rows");
    const uint32_t r = lane >> 4, c = lane & 15u;
#pragma unroll 4
    for (uint32_t s = 0; s < 16; ++s) {
        float av[NT], dv[MT];
#pragma unroll
        for (int n = 0; n < NT; ++n) av[n] = a[4 * s + r][16 * n + c];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            dv[m] = dl[4 * s + r][16 * m + c];
            g.b[m] += dv[m];
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) g.w[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(dv[m], av[n], g.w[m][n], 0, 0, 0);
    }
}

// Adds a wave's layer gradients to gw (W[n_out][n_in], row-major) and gb (b[n_out]).
template <int MT, int NT>
__device__ __forceinline__ void flush(const LayerGrad<MT, NT> &g, float *gw, float *gb, uint32_t n_in,
                                      uint32_t n_out, uint32_t lane)
{
    const uint32_t r = lane >> 4, c = lane & 15u;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t j = 16u * m + 4u * r + k, i = 16u * n + c;
                if (j < n_out && i < n_in) unsafeAtomicAdd(gw + j * n_in + i, g.w[m][n][k]);
            }
        float b = g.b[m];
        b += __shfl_xor(b, 16);
        b += __shfl_xor(b, 32);
        if (r == 0 && 16u * m + c < n_out) unsafeAtomicAdd(gb + 16u * m + c, b);
    }
}


// ---------------------------------------------------------------------------
// the backward's sample order
//
// Texel-gradient float atomics on random lines of levels larger than the
// caches each fetch and write back a whole line. Taking the samples cell by
// cell (and each XCD a contiguous run of cells) lets the samples that share
// gradient lines update them while the lines sit in one L2.

constexpr int kBinThreads = 1024;
// samples a thread of the count and placement kernels takes: a workgroup's
// histogram then covers 16K samples, so that fewer cells of it reach memory
// (one atomic per touched cell and workgroup)
constexpr int kBinPerThread = 16;
constexpr uint32_t kBinPerGroup = kBinThreads * kBinPerThread;

// A query's cell: its wrapped (u, v) on the kTrainBinSide grid (NaN and
// infinities land in cell 0), numbered along a Z-order curve.
__device__ __forceinline__ uint32_t bin_of(float u, float v)
{
    const float uf = u - floorf(u), vf = v - floorf(v);
    const float side = (float)kTrainBinSide;
    const uint32_t cx = (uint32_t)fminf(fmaxf(uf * side, 0.0f), side - 1.0f);
    const uint32_t cy = (uint32_t)fminf(fmaxf(vf * side, 0.0f), side - 1.0f);
    uint32_t z = 0;
#pragma unroll
    for (uint32_t b = 0; b < 6; ++b) z |= ((cx >> b) & 1u) << (2 * b) | ((cy >> b) & 1u) << (2 * b + 1);
    return z;
}

// count[cell] += samples of the cell; kBinPerGroup samples per workgroup
// (sample blockIdx * kBinPerGroup + k * kBinThreads + threadIdx), a histogram in LDS
__global__ void __launch_bounds__(kBinThreads) k_train_bin_count(const float *queries, uint32_t n, uint32_t *count)
{
    __shared__ uint32_t hist[kTrainBins];
    for (uint32_t b = threadIdx.x; b < kTrainBins; b += kBinThreads) hist[b] = 0u;
    __syncthreads();
#pragma unroll 4
    for (uint32_t k = 0; k < (uint32_t)kBinPerThread; ++k) {
        const uint32_t i = blockIdx.x * kBinPerGroup + k * kBinThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[bin_of(queries[3u * i], queries[3u * i + 1u])], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kTrainBins; b += kBinThreads)
        if (hist[b]) atomicAdd(&count[b], hist[b]);
}

// next[cell] = samples of the cells before it (one workgroup, 4 cells a thread)
__global__ void __launch_bounds__(kBinThreads) k_train_bin_scan(const uint32_t *count, uint32_t *next)
{
    static_assert(kTrainBins == 4 * kBinThreads, "four cells a thread");
    __shared__ uint32_t wave_sum[kBinThreads / 64];
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    uint32_t c[4], own = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = count[4 * t + k];
        own += c[k];
    }
    uint32_t incl = own;                           // inclusive scan within the wave
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wave_sum[wv] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t w = 0; w < wv; ++w) base += wave_sum[w];
    uint32_t run = base + incl - own;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        next[4 * t + k] = run;
        run += c[k];
    }
}

// perm[next[cell]++] = sample: each workgroup ranks its kBinPerGroup samples
// (as k_train_bin_count takes them) per cell in LDS, then reserves one run per
// cell it holds
__global__ void __launch_bounds__(kBinThreads) k_train_bin_scatter(const float *queries, uint32_t n, uint32_t *next,
                                                                   uint32_t *perm)
{
    __shared__ uint32_t hist[kTrainBins];
    for (uint32_t b = threadIdx.x; b < kTrainBins; b += kBinThreads) hist[b] = 0u;
    __syncthreads();
    uint32_t bin[kBinPerThread], rank[kBinPerThread];
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kBinPerThread; ++k) {
        const uint32_t i = blockIdx.x * kBinPerGroup + k * kBinThreads + threadIdx.x;
        bin[k] = i < n ? bin_of(queries[3u * i], queries[3u * i + 1u]) : 0u;
        rank[k] = i < n ? atomicAdd(&hist[bin[k]], 1u) : 0u;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kTrainBins; b += kBinThreads)
        if (hist[b]) hist[b] = atomicAdd(&next[b], hist[b]);
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kBinPerThread; ++k) {
        const uint32_t i = blockIdx.x * kBinPerGroup + k * kBinThreads + threadIdx.x;
        if (i < n) perm[hist[bin[k]] + rank[k]] = i;
    }
}

// Y[s][m] = f(sum over k of Wt(m, k) X[s][k] + bias) for the wave's 64
// samples s (rows of the LDS arrays X and Y), m < 16 MT, k < 4 KC, on the
// matrix cores (fp32 16x16x4, K in steps of 4): Wt(m, k) = W[m ldw + k], or
// W[k ldw + m] when TRANS; the bias W[m ldw + bias_col] when BIAS; f = ReLU
// when RELU. Lane L supplies Wt(16 mb + L % 16, 4 kc + L / 16) and X[16 grp
// + L % 16][4 kc + L / 16], and receives rows 4 (L / 16) .. + 3 of sample
// 16 grp + L % 16.
template <int MT, int KC, bool TRANS, bool BIAS, bool RELU, int LDX, int LDY>
__device__ __forceinline__ void rows_product(const float *W, int ldw, int bias_col, const float (*X)[LDX],
                                             float (*Y)[LDY], uint32_t lane)
{
    const uint32_t g = lane >> 4, i16 = lane & 15u;
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
#pragma unroll
        for (int mb = 0; mb < MT; ++mb) {
            f32x4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = BIAS ? W[(16 * mb + 4 * g + r) * ldw + bias_col] : 0.0f;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const uint32_t m = 16 * mb + i16, k = 4 * kc + g;
                const float a = TRANS ? W[k * ldw + m] : W[m * ldw + k];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, X[16 * grp + i16][k], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Y[16 * grp + i16][16 * mb + 4 * g + r] = RELU ? fmaxf(acc[r], 0.0f) : acc[r];
        }
    }
}

// Waves per workgroup of the backward: four when its LDS (per-wave rows for
// the parameter-gradient products, the MLP, the level table) lets two
// workgroups share a CU -- two waves per SIMD, as its registers allow --
// else three.
template <int H, int NH>
constexpr int bwd_waves()
{
    constexpr int rows = 64 * (2 * kTrainMaxHidden + 1) * 4;
    return 4 * rows + (int)sizeof(MlpLds<H, NH>) + (int)sizeof(TrainLevelLut) <= 80 * 1024 ? 4 : 3;
}

template <int H, int NH>
__global__ void __launch_bounds__((64 * bwd_waves<H, NH>()), 2) k_train_backward(TrainDesc d, const float *queries, uint32_t n,
                                                                const float *grad_out, const uint32_t *perm)
{
    constexpr int T = H / 16;                 // 16-wide tiles of a hidden layer
    constexpr int kBwdWaves = bwd_waves<H, NH>();
    __shared__ float lds_a[kBwdWaves][64][kTrainMaxHidden + 1];
    __shared__ float lds_d[kBwdWaves][64][kTrainMaxHidden];
    __shared__ MlpLds<H, NH> mlp;
    __shared__ TrainLevelLut lut;
    load_level_lut(d, lut);
    load_mlp<H, NH>(d, mlp);                  // synchronises, also for `lut`

    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t n0 = d.dims[0], c = d.dims[NH + 1];
    // layer 0 (at most 12 inputs), the hidden layers, the output layer (at most 16 rows)
    LayerGrad<T, 1> g0;
    LayerGrad<T, T> gh[NH > 1 ? NH - 1 : 1];
    LayerGrad<1, T> gl;
    grad_zero(g0);
#pragma unroll
    for (int l = 0; l < (NH > 1 ? NH - 1 : 1); ++l) grad_zero(gh[l]);
    grad_zero(gl);

    float (*a)[kTrainMaxHidden + 1] = lds_a[wv];
    float (*dl)[kTrainMaxHidden] = lds_d[wv];
    // Samples in the sorted order, 64 per wave; workgroups are dealt to the
    // 8 XCDs in turn (the grid is a multiple of 8), and XCD x takes the x-th
    // eighth of the order.
    const uint32_t n_chunks = (n + 63u) / 64u, xcd = blockIdx.x & 7u, xcd_wgs = gridDim.x >> 3;
    const uint32_t c_end = (uint32_t)((uint64_t)n_chunks * (xcd + 1u) / 8u);
    for (uint32_t ch = (uint32_t)((uint64_t)n_chunks * xcd / 8u) + (blockIdx.x >> 3) * kBwdWaves + wv; ch < c_end;
         ch += xcd_wgs * kBwdWaves) {
        const uint32_t slot = ch * 64u + lane;
        const bool live = slot < n;
        const uint32_t q = live ? perm[slot] : 0u;
        const float u = live ? queries[3u * q] : 0.0f;
        const float v = live ? queries[3u * q + 1u] : 0.0f;
        const float s = live ? queries[3u * q + 2u] : 0.0f;
        float z[12], act[NH][H];
        features(d, lut, u, v, s, z);
        // the hidden layers on the matrix cores, layer by layer through the
        // wave's LDS rows (inputs in one array, outputs in the other)
#pragma unroll
        for (int i = 0; i < 12; ++i) a[lane][i] = z[i];
        wave_sync_lds();
        rows_product<T, 3, false, true, true>(&mlp.w0[0][0], 16, 12, a, dl, lane);
        wave_sync_lds();
#pragma unroll
        for (int i = 0; i < H; ++i) act[0][i] = dl[lane][i];
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            if (l & 1) rows_product<T, H / 4, false, true, true>(&mlp.wh[l - 1][0][0], H + 4, H, dl, a, lane);
            else rows_product<T, H / 4, false, true, true>(&mlp.wh[l - 1][0][0], H + 4, H, a, dl, lane);
            wave_sync_lds();
#pragma unroll
            for (int i = 0; i < H; ++i) act[l][i] = l & 1 ? a[lane][i] : dl[lane][i];
            wave_sync_lds();
        }
        float delta[kTrainMaxHidden];
#pragma unroll
        for (int j = 0; j < kTrainMaxHidden; ++j)
            delta[j] = (live && j < kMaxOut && (uint32_t)j < c) ? grad_out[(size_t)q * c + j] : 0.0f;

        // output layer: W[c][H]
#pragma unroll
        for (int i = 0; i < H; ++i) a[lane][i] = act[NH - 1][i];
        a[lane][H] = 1.0f;
#pragma unroll
        for (int j = 0; j < kMaxOut; ++j) dl[lane][j] = delta[j];
        wave_sync_lds();
        accumulate(gl, a, dl, lane);
        wave_sync_lds();
        // back through the hidden layers: delta of hidden layer l's pre-activation
#pragma unroll
        for (int l = NH - 1; l >= 0; --l) {
            // g = W_{l+1}^T delta, summed over the rows j in order; the rows
            // of W_{l+1} are read whole (the output layer's past c are zero,
            // and so are the deltas there)
            // (on the matrix cores: the deltas are dl's rows, the products
            // land in a's rows, which the parameter sums above have read)
            if (l == NH - 1) rows_product<T, kMaxOut / 4, true, false, false>(&mlp.wl[0][0], H + 4, 0, dl, a, lane);
            else rows_product<T, H / 4, true, false, false>(&mlp.wh[l][0][0], H + 4, 0, dl, a, lane);
            wave_sync_lds();
            float g[H];
#pragma unroll
            for (int i = 0; i < H; ++i) g[i] = act[l][i] > 0.0f ? a[lane][i] : 0.0f;
            wave_sync_lds();
#pragma unroll
            for (int i = 0; i < H; ++i) delta[i] = g[i];
            // parameters of layer l: inputs are act[l - 1] (or z), outputs delta
            const uint32_t n_in = l == 0 ? n0 : H;
            if (l == 0) {
#pragma unroll
                for (int i = 0; i < 12; ++i) a[lane][i] = z[i];
            } else {
#pragma unroll
                for (int i = 0; i < H; ++i) a[lane][i] = act[l > 0 ? l - 1 : 0][i];
            }
            a[lane][n_in] = 1.0f;
#pragma unroll
            for (int j = 0; j < H; ++j) dl[lane][j] = delta[j];
            wave_sync_lds();
            if (l == 0) accumulate(g0, a, dl, lane);
            else accumulate(gh[l > 0 ? l - 1 : 0], a, dl, lane);
            wave_sync_lds();
        }
        // dL/dz = W_0^T delta (rows 12 .. 15 of the product, from the bias
        // column and the padding, are not used)
        rows_product<1, H / 4, true, false, false>(&mlp.w0[0][0], 16, 0, dl, a, lane);
        wave_sync_lds();
        float dz[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) dz[i] = a[lane][i];
        wave_sync_lds();
        // dL/dz in the sorted order, for the scatter
        if (live) {
            float4 *dst = reinterpret_cast<float4 *>(d.bin_dz + 12u * (size_t)slot);
            dst[0] = make_float4(dz[0], dz[1], dz[2], dz[3]);
            dst[1] = make_float4(dz[4], dz[5], dz[6], dz[7]);
            dst[2] = make_float4(dz[8], dz[9], dz[10], dz[11]);
        }
    }
    flush(g0, d.g_params + d.w_off[0], d.g_params + d.b_off[0], n0, H, lane);
#pragma unroll
    for (int l = 1; l < NH; ++l) flush(gh[l - 1], d.g_params + d.w_off[l], d.g_params + d.b_off[l], H, H, lane);
    flush(gl, d.g_params + d.w_off[NH], d.g_params + d.b_off[NH], H, c, lane);
}

// ---------------------------------------------------------------------------
// dL/dz -> dL/d texel

constexpr int kScatterThreads = 256;
constexpr uint32_t kWindowFloats = 8192;      // 32 KB of LDS windows per workgroup

// A window of one (pyramid, level): the texels x0 .. x0 + w - 1 (wrapped) of
// rows y0 .. y0 + h - 1, three floats each from `off` in the pool; off = ~0u:
// the level's gradients go straight to memory. div_w = ceil(2^32 / w) (w > 1),
// so that p / w = umulhi(p, div_w) for the pool's positions p (p < 2^13).
struct TexWindow {
    uint32_t x0, y0, w, h, off, div_w;
};

// One workgroup per cell of the sample sort: the cell's samples (sorted
// indices begin .. end) add wt * dL/dz to the texels of their taps. Every tap
// of a cell's samples at one (pyramid, level) lies in a small box around the
// cell's footprint, so the sums go to LDS windows over those boxes (the
// coarsest levels first, while the pool lasts) and then to memory once per
// touched texel channel; a tap outside its window (or of a level without one)
// goes to memory directly.
__global__ void __launch_bounds__(kScatterThreads) k_train_scatter(TrainDesc d, const float *queries)
{
    __shared__ float pool[kWindowFloats];
    __shared__ TexWindow win[kMaxTextures][kMaxLevels];
    __shared__ TrainLevelLut lut;
    __shared__ uint32_t pool_used, dz_max_bits;
    const uint32_t cell = blockIdx.x;
    const uint32_t begin = cell ? d.bin_next[cell - 1] : 0u, end = d.bin_next[cell];
    if (begin == end) return;                          // uniform over the workgroup
    load_level_lut(d, lut);
    __syncthreads();
    if (threadIdx.x < 64u) {
        // lane i: window i of the allocation order, the coarsest levels first
        // (level 15 - i / 4, pyramid i % 4); the pool goes to a prefix of it
        const uint32_t i = threadIdx.x, l = kMaxLevels - 1u - i / kMaxTextures, t = i % kMaxTextures;
        static_assert(kMaxLevels * kMaxTextures == 64, "one lane per window");
        // the cell's corner from its Z-order number
        uint32_t cx = 0, cy = 0;
#pragma unroll
        for (uint32_t b = 0; b < 6; ++b) {
            cx |= ((cell >> (2 * b)) & 1u) << b;
            cy |= ((cell >> (2 * b + 1)) & 1u) << b;
        }
        const uint32_t levels_t = t == 0 ? d.tex[0].levels : t == 1 ? d.tex[1].levels
                                : t == 2 ? d.tex[2].levels : d.tex[3].levels;
        const bool have = t < d.n_tex && l < levels_t;
        // a cell spans wl / side texels; its samples' taps span at most ceil
        // of that + 2 columns from floor(cx wl / side - 0.5)
        const uint32_t wl = lut[t][l].x, hl = lut[t][l].y;
        const uint32_t ww = min(wl, (wl + kTrainBinSide - 1) / kTrainBinSide + 2u);
        const uint32_t wh = min(hl, (hl + kTrainBinSide - 1) / kTrainBinSide + 2u);
        const uint32_t size = have ? 3u * ww * wh : 0u;
        uint32_t upto = size;                      // inclusive prefix over the order
#pragma unroll
        for (uint32_t k = 1; k < 64; k <<= 1) {
            const uint32_t o = __shfl_up(upto, k);
            if (i >= k) upto += o;
        }
        const float fx = floorf((float)cx * ((float)wl / (float)kTrainBinSide) - 0.5f);
        const float fy = floorf((float)cy * ((float)hl / (float)kTrainBinSide) - 0.5f);
        TexWindow W;
        W.x0 = ww == wl ? 0u : (uint32_t)(int)fx & (wl - 1u);
        W.y0 = wh == hl ? 0u : (uint32_t)(int)fy & (hl - 1u);
        W.w = ww;
        W.h = wh;
        W.off = have && upto <= kWindowFloats ? upto - size : ~0u;
        W.div_w = ww > 1u ? 0xFFFFFFFFu / ww + 1u : 0u;
        win[t][l] = W;
        // the pool in use: the end of the last window that fits
        uint32_t in_use = upto <= kWindowFloats ? upto : 0u;
#pragma unroll
        for (uint32_t k = 1; k < 64; k <<= 1) in_use = max(in_use, __shfl_xor(in_use, k));
        if (i == 0u) pool_used = in_use;
    }
    // The largest |dL/dz| of the cell's samples (as bits: NaN and infinity
    // above every finite value) sets the windows' fixed-point scale.
    if (threadIdx.x == 0) dz_max_bits = 0u;
    __syncthreads();
    {
        uint32_t mb = 0;
        for (uint32_t j = begin + threadIdx.x; j < end; j += kScatterThreads) {
            const uint4 *src = reinterpret_cast<const uint4 *>(d.bin_dz + 12u * (size_t)j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint4 z = src[k];
                mb = max(mb, max(max(z.x & 0x7FFFFFFFu, z.y & 0x7FFFFFFFu), max(z.z & 0x7FFFFFFFu, z.w & 0x7FFFFFFFu)));
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mb = max(mb, (uint32_t)__shfl_xor((int)mb, o));
        if ((threadIdx.x & 63u) == 0) atomicMax(&dz_max_bits, mb);
    }
    const uint32_t used = pool_used;
    for (uint32_t e = threadIdx.x; e < used; e += kScatterThreads) pool[e] = 0.0f;
    __syncthreads();
    // LDS float atomics cost about 40 times integer ones on this GPU, so the
    // windows sum in 32-bit fixed point: contribution v adds rint(v 2^k),
    // with 2^k chosen so that the at most nc M of a texel channel (nc samples,
    // each adding at most M = max |dL/dz| over its taps, whose weights sum to
    // at most 1) stays below 2^29. Non-finite gradients take float atomics.
    const uint32_t mbits = dz_max_bits;
    const bool fixed = mbits < 0x7F800000u;
    int kexp = 0;
    if (fixed && mbits != 0u) {
        int em;
        frexpf(__uint_as_float(mbits), &em);                  // M < 2^em
        const uint32_t nc = end - begin;
        const int en = 32 - __clz(nc);                       // nc < 2^en
        kexp = min(max(29 - em - en, -120), 120);
    }
    const float scale = ldexpf(1.0f, kexp), unscale = ldexpf(1.0f, -kexp);
    for (uint32_t j = begin + threadIdx.x; j < end; j += kScatterThreads) {
        const uint32_t q = d.bin_perm[j];
        const float4 *src = reinterpret_cast<const float4 *>(d.bin_dz + 12u * (size_t)j);
        const float4 z0 = src[0], z1 = src[1], z2 = src[2];
        const float dz[12] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w, z2.x, z2.y, z2.z, z2.w};
        const float u = queries[3u * q], v = queries[3u * q + 1u], s = queries[3u * q + 2u];
        const float uf = u - floorf(u), vf = v - floorf(v);       // wrap addressing
#pragma unroll
        for (int t = 0; t < kMaxTextures; ++t) {
            if (t >= (int)d.n_tex) break;
            // the two levels of eq. (10) as the forward takes them
            const TrainTexDesc &tx = d.tex[t];
            const float si = fminf(fmaxf(s + tx.bias, 0.0f), (float)(tx.levels - 1));   // NaN -> 0
            const uint32_t l0 = (uint32_t)floorf(si);
            const uint32_t l1 = min(l0 + 1u, tx.levels - 1u);
            const float lam = si - (float)l0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t l = k ? l1 : l0;
                const float lw = k ? lam : 1.0f - lam;
                // a zero weight (an unused second level) adds nothing
                if (lw == 0.0f) continue;
                const uint4 e = lut[t][l];
                const LevelTaps lt = level_taps(e, uf, vf, lw);
                const TexWindow W = win[t][l];
                const uint32_t dxa = (lt.xa - W.x0) & (e.x - 1u), dxb = (lt.xb - W.x0) & (e.x - 1u);
                const uint32_t dya = (lt.ya - W.y0) & (e.y - 1u), dyb = (lt.yb - W.y0) & (e.y - 1u);
                const uint32_t base = W.off;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float wt = lt.w[i];
                    if (wt == 0.0f) continue;
                    const uint32_t x = i & 1 ? lt.xb : lt.xa, y = i & 2 ? lt.yb : lt.ya;
                    const uint32_t dx = i & 1 ? dxb : dxa, dy = i & 2 ? dyb : dya;
                    if (W.off != ~0u && dx < W.w && dy < W.h) {
                        float *p = pool + base + 3u * (__umul24(dy, W.w) + dx);
                        if (fixed) {
                            uint32_t *pi = reinterpret_cast<uint32_t *>(p);
#pragma unroll
                            for (int c = 0; c < 3; ++c)
                                atomicAdd(pi + c, (uint32_t)(int32_t)rintf(wt * dz[3 * t + c] * scale));
                        } else {
#pragma unroll
                            for (int c = 0; c < 3; ++c) atomicAdd(p + c, wt * dz[3 * t + c]);
                        }
                    } else {
                        float *gp = reinterpret_cast<float *>(d.g_texels + e.z + y * e.x + x);
                        unsafeAtomicAdd(gp + 0, wt * dz[3 * t + 0]);
                        unsafeAtomicAdd(gp + 1, wt * dz[3 * t + 1]);
                        unsafeAtomicAdd(gp + 2, wt * dz[3 * t + 2]);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t t = 0; t < d.n_tex; ++t)
        for (uint32_t l = 0; l < d.tex[t].levels; ++l) {
            const TexWindow W = win[t][l];
            if (W.off == ~0u) continue;
            const uint4 e = lut[t][l];
            const uint32_t size = 3u * W.w * W.h;
            for (uint32_t i = threadIdx.x; i < size; i += kScatterThreads) {
                const float raw = pool[W.off + i];
                const float v = fixed ? (float)__float_as_int(raw) * unscale : raw;
                if (v == 0.0f) continue;
                const uint32_t p = i / 3u, c = i - 3u * p, dy = W.w > 1u ? __umulhi(p, W.div_w) : p, dx = p - dy * W.w;
                const uint32_t x = (W.x0 + dx) & (e.x - 1u), y = (W.y0 + dy) & (e.y - 1u);
                unsafeAtomicAdd(reinterpret_cast<float *>(d.g_texels + e.z + y * e.x + x) + c, v);
            }
        }
}

unsigned grid_for(size_t work, unsigned per_block, unsigned cap)
{
    const size_t g = (work + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_texels(const TrainDesc &d, hipStream_t s)
{
    const unsigned grid = grid_for((size_t)d.blk_base[d.n_tex] * 4u, kTrainThreads, 16384);
    if (d.ste) k_train_texels<true><<<grid, kTrainThreads, 0, s>>>(d);
    else k_train_texels<false><<<grid, kTrainThreads, 0, s>>>(d);
    return hipGetLastError();
}

template <int H, int NH>
hipError_t forward_hn(const TrainDesc &d, const float *queries, uint32_t n, float *out, hipStream_t s)
{
    hipError_t e = launch_prepare_weights(d.params, nullptr, d.ops_shape, MLP_MFMA_F32, d.ops, d.ops_ws, nullptr, s);
    if (e != hipSuccess) return e;
    k_train_forward_mfma<H, NH><<<grid_for(n, kTrainThreads, 8192), kTrainThreads, 0, s>>>(d, queries, n, out);
    return hipGetLastError();
}

template <int H, int NH>
hipError_t backward_hn(const TrainDesc &d, const float *queries, uint32_t n, const float *grad_out, hipStream_t s)
{
    // a few workgroups per CU (each flushes its parameter and small-level
    // sums once), a multiple of the 8 XCDs
    constexpr int waves = bwd_waves<H, NH>();
    const unsigned grid = (grid_for((n + 63u) / 64u, waves, 768) + 7u) & ~7u;
    k_train_backward<H, NH><<<grid, 64 * waves, 0, s>>>(d, queries, n, grad_out, d.bin_perm);
    return hipGetLastError();
}

#define BCF_TRAIN_DISPATCH(fn, ...)                                                           \
    do {                                                                                      \
        const uint32_t H = d.dims[1], NH = d.n_layers - 1;                                    \
        if (H == 16 && NH == 1) return fn<16, 1>(d, __VA_ARGS__);                             \
        if (H == 16 && NH == 2) return fn<16, 2>(d, __VA_ARGS__);                             \
        if (H == 16 && NH == 3) return fn<16, 3>(d, __VA_ARGS__);                             \
        if (H == 32 && NH == 1) return fn<32, 1>(d, __VA_ARGS__);                             \
        if (H == 32 && NH == 2) return fn<32, 2>(d, __VA_ARGS__);                             \
        if (H == 32 && NH == 3) return fn<32, 3>(d, __VA_ARGS__);                             \
        return hipErrorInvalidValue;                                                          \
    } while (0)

hipError_t dispatch_forward(const TrainDesc &d, const float *queries, uint32_t n, float *out, hipStream_t s)
{
    BCF_TRAIN_DISPATCH(forward_hn, queries, n, out, s);
}

hipError_t dispatch_backward(const TrainDesc &d, const float *queries, uint32_t n, const float *grad_out,
                             hipStream_t s)
{
    BCF_TRAIN_DISPATCH(backward_hn, queries, n, grad_out, s);
}

#undef BCF_TRAIN_DISPATCH

}  // namespace

hipError_t launch_train_forward(const TrainDesc &d, const float *queries, size_t n, float *out, hipStream_t s)
{
    hipError_t e = launch_texels(d, s);
    if (e != hipSuccess || n == 0) return e;
    return dispatch_forward(d, queries, (uint32_t)n, out, s);
}

hipError_t launch_train_backward(const TrainDesc &d, const float *queries, size_t n, const float *grad_out,
                                 hipStream_t s)
{
    hipError_t e = launch_texels(d, s);
    if (e != hipSuccess) return e;
    k_train_zero<<<grid_for((size_t)d.n_texels * 4u, 256, 8192), 256, 0, s>>>(
        reinterpret_cast<float *>(d.g_texels), d.n_texels * 4u);
    k_train_zero<<<grid_for(d.n_params, 256, 64), 256, 0, s>>>(d.g_params, d.n_params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint32_t c = d.dims[d.n_layers];
    for (size_t off = 0; off < n; off += kTrainBinBatch) {
        const uint32_t m = (uint32_t)std::min(n - off, (size_t)kTrainBinBatch);
        const float *q = queries + 3 * off;
        const unsigned bins = (m + kBinPerGroup - 1) / kBinPerGroup;
        // (the counts are cleared as floats: 0.0f is all zero bits)
        k_train_zero<<<8, 256, 0, s>>>(reinterpret_cast<float *>(d.bin_count), kTrainBins);
        k_train_bin_count<<<bins, kBinThreads, 0, s>>>(q, m, d.bin_count);
        k_train_bin_scan<<<1, kBinThreads, 0, s>>>(d.bin_count, d.bin_next);
        k_train_bin_scatter<<<bins, kBinThreads, 0, s>>>(q, m, d.bin_next, d.bin_perm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = dispatch_backward(d, q, m, grad_out + (size_t)c * off, s)) != hipSuccess) return e;
        k_train_scatter<<<kTrainBins, kScatterThreads, 0, s>>>(d, q);
    }
    const unsigned grid = grid_for((size_t)d.blk_base[d.n_tex] * 16u, kTrainThreads, 16384);
    if (d.ste) k_train_blocks<true><<<grid, kTrainThreads, 0, s>>>(d);
    else k_train_blocks<false><<<grid, kTrainThreads, 0, s>>>(d);
    return hipGetLastError();
}

}  // namespace bcf
