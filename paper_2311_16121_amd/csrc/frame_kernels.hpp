// The decode and calibration kernels, instantiated per MLP precision in
// frame_<precision>.hip (separate translation units compile in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "filter_device.hpp"
#include "internal.hpp"
#include "mlp_device.hpp"

namespace bcf {

typedef uint32_t uint4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// The decode kernel: one query per lane filters the four pyramid slots, then
// the MLP:
//  * plain fp32: in the lane, with wave-uniform (scalar) weight operands;
//  * MFMA: the wave's 64 feature vectors go through LDS into the operand
//    layout of mlp_device.hpp, four groups of 16 queries per wave.
// Outputs are staged in LDS so each wave writes its 64 rows as contiguous
// 16-byte stores.

constexpr int kFrameThreads = 256;
constexpr int kFrameWaves = kFrameThreads / 64;
// 16-byte output chunks per lane of a 64-query item (64 rows of <= 16 floats)
constexpr int kTileChunks = 64 * kMaxOut / 4 / 64;

// a wave's 64 feature vectors (4 x float4 each) fit its output stage
static_assert(64 * 4 <= 64 * kMaxOut / 4, "feature vectors must fit the output stage");

struct FrameArgs {
    LevelLut lut;
    float levels_bias[2 * kMaxTextures];   // per slot: level count (bits), b_i
    uint32_t stride;                       // shared geometry: bytes between slots' scratch
    const uint8_t *ws;
    WsLayout lay;
    const float *queries;
    float *out;
    uint32_t n;                            // queries of this launch
    uint32_t out_dim;
    float *absmax;                         // k_calibrate: per-layer largest |input|
    // 2D work items: with grid_w > 0 the queries are image rows of grid_w and
    // a wave takes a tile of 2^tile_log2 columns by 64 / 2^tile_log2 rows
    // (lane = row * width + column); with 0, 64 consecutive queries.
    // rows_b128: grid_w * out_dim is a multiple of 4 (16-byte rows)
    uint32_t grid_w, tiles_x, n_items, rows_b128, tile_log2;
};

// The grid is a multiple of the 8 XCDs (workgroups are dispatched to them
// round-robin). Work items go round-robin over all waves, so the waves on the
// chip at any moment work on neighbouring items (measured faster than giving
// each XCD its own band: the bands differ in how often they miss L2).
constexpr uint32_t kXcds = 8;

struct ItemRange {
    uint32_t first, end, step;
};

__device__ __forceinline__ ItemRange wave_items(uint32_t n_items, uint32_t wv)
{
    return ItemRange{blockIdx.x * kFrameWaves + wv, n_items, gridDim.x * kFrameWaves};
}

struct Query {
    float u, v, s;
};

// One 12-byte query through the buffer descriptor (reads past the end give 0).
// The vector's elements go through plain integers before the bit casts.
__device__ __forceinline__ Query load_query(__amdgpu_buffer_rsrc_t rq, uint32_t q)
{
    const auto qv = __builtin_amdgcn_raw_buffer_load_b96(rq, (int)(q * 12u), 0, 0);
    const uint32_t u = qv[0], v = qv[1], s = qv[2];
    return Query{__builtin_bit_cast(float, u), __builtin_bit_cast(float, v), __builtin_bit_cast(float, s)};
}

// The MLP parameters do not change during a launch: reading them through the
// constant address space lets the compiler use scalar loads and SGPR operands.
typedef const __attribute__((address_space(4))) float const_float;

__device__ __forceinline__ const_float *constant_floats(const uint8_t *p)
{
    return (const_float *)p;
}

// Row j of a layer's weights and its bias, through the constant address
// space (scalar loads, SGPR operands). The pointer goes through an empty asm
// per row, so the optimiser can neither hoist the loads out of the caller's
// query loop nor keep more than about a row's weights live: 1-2k weights do
// not fit in SGPRs and would be spilled.
__device__ __forceinline__ const_float *weight_row(const uint8_t *ws, size_t off, uint32_t row, uint32_t n_in)
{
    asm volatile("" : "+s"(ws));
    return constant_floats(ws + off) + row * n_in;
}

template <int N_IN>
__device__ __forceinline__ float neuron(const uint8_t *ws, const WsLayout &lay, int l, uint32_t j, const float *x)
{
    const_float *w = weight_row(ws, lay.layer_w_off[l], j, N_IN);
    float acc = constant_floats(ws + lay.layer_b_off[l])[j];
#pragma unroll
    for (int i = 0; i < N_IN; ++i) acc = fmaf(w[i], x[i], acc);
    return acc;
}

template <int H, int NH, int C>
__device__ __forceinline__ void mlp_valu(const uint8_t *ws, const WsLayout &lay, const float z[12], float o[C],
                                         float *amax)
{
    if (amax) {
#pragma unroll
        for (int i = 0; i < 12; ++i) amax[0] = fmaxf(amax[0], fabsf(z[i]));
    }
    float hcur[H];
#pragma unroll
    for (int j = 0; j < H; ++j) hcur[j] = relu(neuron<12>(ws, lay, 0, j, z));
#pragma unroll
    for (int l = 1; l < NH; ++l) {
        if (amax) {
#pragma unroll
            for (int i = 0; i < H; ++i) amax[l] = fmaxf(amax[l], hcur[i]);
        }
        float hn[H];
#pragma unroll
        for (int j = 0; j < H; ++j) hn[j] = relu(neuron<H>(ws, lay, l, j, hcur));
#pragma unroll
        for (int j = 0; j < H; ++j) hcur[j] = hn[j];
    }
    if (amax) {
#pragma unroll
        for (int i = 0; i < H; ++i) amax[NH] = fmaxf(amax[NH], hcur[i]);
    }
#pragma unroll
    for (int j = 0; j < C; ++j) o[j] = neuron<H>(ws, lay, NH, j, hcur);
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void copy_lut(const LevelLut &src, LevelLut &dst)
{
    const uint4 *s = &src.e[0][0];
    uint4 *d = &dst.e[0][0];
    for (int i = threadIdx.x; i < kMaxTextures * kMaxLevels; i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

// MLP (eq. 3) of a wave's 64 feature vectors z (one per lane); the outputs
// land in the wave's LDS stage, lane L's at st[L * out_dim ...]. The MFMA path
// passes the feature vectors through `feats`, which may be the same LDS as st
// (both 4 KB).
template <MlpKind K, int H, int NH, int C>
__device__ __forceinline__ void mlp_stage(const float z[12], const uint8_t *wbase, const WsLayout &lay,
                                          const MfmaMlp<K == MLP_VALU_F32 ? MLP_MFMA_F16 : K, H, NH> &mlp,
                                          float4_t (*feats)[4], float *st, uint32_t out_dim, uint32_t lane)
{
    constexpr bool VALU = K == MLP_VALU_F32;
    const uint32_t g = lane >> 4, qi = lane & 15;
    if (VALU) {
        float o[C];
        mlp_valu<H, NH, C>(wbase, lay, z, o, nullptr);
#pragma unroll
        for (int j = 0; j < C; ++j)
            if ((uint32_t)j < out_dim) st[lane * out_dim + j] = o[j];
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float4_t v4 = {z[3 * t], z[3 * t + 1], z[3 * t + 2], 0.0f};
            feats[lane][t] = v4;
        }
        wave_lds_sync();
        float4_t fin[4];
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) fin[grp] = feats[16 * grp + qi][g];
        wave_lds_sync();                      // feats and st share the wave's LDS
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            const float f[4] = {fin[grp][0], fin[grp][1], fin[grp][2], fin[grp][3]};
            const float4_t o4 = mlp.run(f);
            const uint32_t row = (16 * grp + qi) * out_dim;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * g + j < out_dim) st[row + 4 * g + j] = o4[j];
        }
    }
    wave_lds_sync();
}

// One wave's 64 queries: filter (eqs. 9, 10), concatenate, MLP.
template <MlpKind K, int H, int NH, int C, bool SHARED>
__device__ __forceinline__ void decode_wave(const Query &qq, __amdgpu_buffer_rsrc_t rs, const LevelLut &lut,
                                            const float *levels_bias, uint32_t stride, const uint8_t *wbase,
                                            const WsLayout &lay,
                                            const MfmaMlp<K == MLP_VALU_F32 ? MLP_MFMA_F16 : K, H, NH> &mlp,
                                            float4_t (*feats)[4], float *st, uint32_t out_dim, uint32_t lane)
{
    float z[12];
    filter4<SHARED>(rs, lut, levels_bias, stride, qq.u, qq.v, qq.s, z);
    mlp_stage<K, H, NH, C>(z, wbase, lay, mlp, feats, st, out_dim, lane);
}

// Item `it` of a run of n consecutive queries: its (up to) 64 staged rows go
// to out as 16-byte stores, the last partial item as 4-byte stores.
__device__ __forceinline__ void store_run(const float4_t *stage, __amdgpu_buffer_rsrc_t ro, uint32_t it, uint32_t n,
                                          uint32_t out_dim, uint32_t lane)
{
    const uint32_t base = it * 64u * out_dim * 4u;
    if (it * 64 + 64 <= n) {
        for (uint32_t k = lane; k < 16 * out_dim; k += 64)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4_t, stage[k]), ro, (int)(base + 16u * k),
                                                   0, 0);
    } else {
        const float *st = reinterpret_cast<const float *>(stage);
        const uint32_t floats = (n - it * 64) * out_dim;
        for (uint32_t k = lane; k < floats; k += 64)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, st[k]), ro, (int)(base + 4u * k), 0,
                                                  0);
    }
}

template <MlpKind K, int H, int NH, int C, bool SHARED>
__global__ void __launch_bounds__(kFrameThreads) k_frame(FrameArgs a)
{
    constexpr bool VALU = K == MLP_VALU_F32;
    __shared__ LevelLut lut;
    // per wave 4 KB: the feature vectors, then the staged output rows
    __shared__ float4_t stage[kFrameWaves][64 * kMaxOut / 4];
    copy_lut(a.lut, lut);

    // the wave index is uniform across the wave: say so, so that everything
    // derived from it (work items, materials, offsets) lives in SGPRs
    const uint32_t lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ws + a.lay.scratch_off, (uint32_t)a.lay.scratch_bytes);
    const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.queries, a.n * 12u);
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out, a.n * a.out_dim * 4u);
    MfmaMlp<VALU ? MLP_MFMA_F16 : K, H, NH> mlp;
    if (!VALU) mlp.load(a.ws, a.lay, lane);
    float *st = reinterpret_cast<float *>(&stage[wv][0]);
    float4_t (*feats)[4] = reinterpret_cast<float4_t (*)[4]>(&stage[wv][0]);

    // Full tiles store each row of tile_w * out_dim floats as 16-byte chunks;
    // chunk k = lane + 64 m sits at tile_off[m] bytes from the tile's first
    // output (all-ones: no such chunk).
    const uint32_t tile_w = 1u << a.tile_log2, tile_h = 64u >> a.tile_log2;
    uint32_t tile_off[kTileChunks];
    {
        const uint32_t per_row = (tile_w * a.out_dim) >> 2;
#pragma unroll
        for (int m = 0; m < kTileChunks; ++m) {
            const uint32_t k = lane + 64u * m, r = k / per_row, c = k - r * per_row;
            tile_off[m] = k < 16u * a.out_dim ? r * a.grid_w * a.out_dim * 4u + 16u * c : 0xFFFFFFFFu;
        }
    }
    // this lane's query of item `it` (and the item's tile origin); lanes
    // outside the image or past n read zeros (buffer range check) and their
    // rows are not stored
    auto query_of = [&](uint32_t it, uint32_t &row0, uint32_t &col0) -> uint32_t {
        if (!a.grid_w) {
            row0 = col0 = 0;
            return it * 64 + lane;
        }
        row0 = (it / a.tiles_x) * tile_h;
        col0 = (it % a.tiles_x) * tile_w;
        const uint32_t col = col0 + (lane & (tile_w - 1u));
        const uint32_t q = (row0 + (lane >> a.tile_log2)) * a.grid_w + col;
        return col < a.grid_w && q < a.n ? q : a.n;
    };
    const ItemRange items = wave_items(a.n_items, wv);
    uint32_t row0, col0;
    // the next item's query is loaded while this item's texels are fetched
    Query next = load_query(rq, query_of(items.first < items.end ? items.first : 0, row0, col0));
    for (uint32_t it = items.first; it < items.end; it += items.step) {
        query_of(it, row0, col0);
        const Query qq = next;
        if (it + items.step < items.end) {
            uint32_t r, c;
            next = load_query(rq, query_of(it + items.step, r, c));
        }
        decode_wave<K, H, NH, C, SHARED>(qq, rs, lut, a.levels_bias, a.stride, a.ws, a.lay, mlp, feats, st,
                                         a.out_dim, lane);
        // Staged rows: lane L's outputs at st[L * out_dim ...]. A tile row or a
        // run of 64 consecutive queries is one contiguous span of out.
        if (!a.grid_w) {
            store_run(stage[wv], ro, it, a.n, a.out_dim, lane);
        } else {
            const bool full = col0 + tile_w <= a.grid_w && (row0 + tile_h - 1u) * a.grid_w + col0 + tile_w <= a.n;
            if (full && a.rows_b128) {
                const uint32_t base = (row0 * a.grid_w + col0) * a.out_dim * 4u;
#pragma unroll
                for (int m = 0; m < kTileChunks; ++m)
                    if (tile_off[m] != 0xFFFFFFFFu)
                        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4_t, stage[wv][lane + 64 * m]),
                                                               ro, (int)(base + tile_off[m]), 0, 0);
            } else {                                   // an edge tile
                for (uint32_t k = lane; k < 64u * a.out_dim; k += 64) {
                    const uint32_t src = k / a.out_dim, j = k - src * a.out_dim;
                    const uint32_t col = col0 + (src & (tile_w - 1u));
                    const uint32_t qq2 = (row0 + (src >> a.tile_log2)) * a.grid_w + col;
                    if (col < a.grid_w && qq2 < a.n)
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, st[k]), ro,
                                                              (int)((qq2 * a.out_dim + j) * 4u), 0, 0);
                }
            }
        }
        wave_lds_sync();
    }
}

// The plain fp32 decode that records each layer's largest input magnitude
// (the static fp8 activation scales come from a calibration batch).
template <int H, int NH, int C, bool SHARED>
__global__ void __launch_bounds__(kFrameThreads) k_calibrate(FrameArgs a)
{
    __shared__ LevelLut lut;
    copy_lut(a.lut, lut);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ws + a.lay.scratch_off, (uint32_t)a.lay.scratch_bytes);
    const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.queries, a.n * 12u);
    float amax[NH + 1];
#pragma unroll
    for (int l = 0; l <= NH; ++l) amax[l] = 0.0f;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < a.n; q += gridDim.x * blockDim.x) {
        const Query qq = load_query(rq, q);
        float z[12], o[C];
        filter4<SHARED>(rs, lut, a.levels_bias, a.stride, qq.u, qq.v, qq.s, z);
        mlp_valu<H, NH, C>(a.ws, a.lay, z, o, amax);
    }
#pragma unroll
    for (int l = 0; l <= NH; ++l) {
        // non-negative floats order like their bit patterns
        atomicMax(reinterpret_cast<unsigned int *>(a.absmax) + l, __builtin_bit_cast(unsigned int, amax[l]));
    }
}




// ---------------------------------------------------------------------------
// Many materials in one launch. Every material has its own pyramids, texel
// scratch and MLP weights (one MLP shape for all); its queries are a
// contiguous range of the concatenated query array. Work items are runs of 64
// queries of one material, numbered material after material.

// A wave-uniform value loaded from memory, moved to SGPRs.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

struct BatchMat {
    LevelLut lut;                          // as FrameArgs, offsets within the material's scratch
    float levels_bias[2 * kMaxTextures];
    uint64_t scratch_off, weights_off;     // bytes from the workspace start
    uint32_t scratch_bytes, stride, shared, pad;
};

struct BatchArgs {
    const uint8_t *ws;
    const BatchMat *mats;                  // [n_mats], in the workspace
    const uint32_t *offsets;               // caller's [n_mats + 1] first query of each material
    uint32_t *items;                       // [n_mats + 1] first item of each material (k_batch_items)
    WsLayout lay;                          // weight layout relative to a material's weights_off
    const float *queries;
    float *out;
    uint32_t n_mats, n_total, out_dim;
    uint32_t interleave;                   // 1: waves of an XCD interleave items; 0: contiguous ranges
};

// Query range of material k: the caller's offsets clamped to [0, n_total],
// made non-decreasing, at most kMaxQueriesPerLaunch queries.
__device__ __forceinline__ void batch_range(const BatchArgs &a, uint32_t k, uint32_t &q0, uint32_t &cnt)
{
    q0 = min(a.offsets[k], a.n_total);
    const uint32_t q1 = max(min(a.offsets[k + 1], a.n_total), q0);
    cnt = min(q1 - q0, (uint32_t)kMaxQueriesPerLaunch);
}

template <MlpKind K, int H, int NH, int C>
__global__ void __launch_bounds__(kFrameThreads) k_batch(BatchArgs a)
{
    constexpr bool VALU = K == MLP_VALU_F32;
    __shared__ LevelLut lut[kFrameWaves];                 // each wave's current material
    __shared__ float4_t stage[kFrameWaves][64 * kMaxOut / 4];   // features, then output rows
    // the wave index is uniform across the wave: say so, so that everything
    // derived from it (work items, materials, offsets) lives in SGPRs
    const uint32_t lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *st = reinterpret_cast<float *>(&stage[wv][0]);
    float4_t (*feats)[4] = reinterpret_cast<float4_t (*)[4]>(&stage[wv][0]);
    const uint32_t total = a.items[a.n_mats];

    ItemRange items;
    if (a.interleave) {
        items = wave_items(total, wv);
    } else {
        // contiguous: the XCD's band split into one range per wave
        const uint32_t xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
        const uint32_t waves = (gridDim.x / kXcds) * kFrameWaves, w = local * kFrameWaves + wv;
        const uint64_t lo = (uint64_t)total * xcd / kXcds, hi = (uint64_t)total * (xcd + 1) / kXcds;
        items.first = (uint32_t)(lo + (hi - lo) * w / waves);
        items.end = (uint32_t)(lo + (hi - lo) * (w + 1) / waves);
        items.step = 1;
    }

    MfmaMlp<VALU ? MLP_MFMA_F16 : K, H, NH> mlp;
    uint32_t cur = 0xFFFFFFFFu, first_item = 0, n_k = 0, shared = 0, stride = 0;
    float lb[2 * kMaxTextures];
    const uint8_t *wbase = a.ws;
    __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ws, 0), rq = rs, ro = rs;
    for (uint32_t it = items.first; it < items.end; it += items.step) {
        // the material: the last k with items[k] <= it (empty materials share
        // their first item with the next one, which the search lands on)
        uint32_t lo = 0, hi = a.n_mats;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.items[mid] <= it) lo = mid;
            else hi = mid;
        }
        lo = uniform(lo);
        if (lo != cur) {
            cur = lo;
            const BatchMat &M = a.mats[cur];
            lut[wv].e[lane >> 4][lane & 15] = M.lut.e[lane >> 4][lane & 15];
#pragma unroll
            for (int j = 0; j < 2 * kMaxTextures; ++j)
                lb[j] = __builtin_bit_cast(float, uniform(__builtin_bit_cast(uint32_t, M.levels_bias[j])));
            shared = uniform(M.shared);
            stride = uniform(M.stride);
            rs = make_rsrc(a.ws + uniform64(M.scratch_off), uniform(M.scratch_bytes));
            uint32_t q0;
            batch_range(a, cur, q0, n_k);
            q0 = uniform(q0);
            n_k = uniform(n_k);
            rq = make_rsrc(a.queries + 3ull * q0, n_k * 12u);
            ro = make_rsrc(a.out + (uint64_t)a.out_dim * q0, n_k * a.out_dim * 4u);
            wbase = a.ws + uniform64(M.weights_off);
            if (!VALU) mlp.load(wbase, a.lay, lane);
            first_item = uniform(a.items[cur]);
            wave_lds_sync();
        }
        const uint32_t j = it - first_item;
        const Query qq = load_query(rq, j * 64 + lane);   // past n_k: zeros, not stored
        if (shared)
            decode_wave<K, H, NH, C, true>(qq, rs, lut[wv], lb, stride, wbase, a.lay, mlp, feats, st,
                                           a.out_dim, lane);
        else
            decode_wave<K, H, NH, C, false>(qq, rs, lut[wv], lb, stride, wbase, a.lay, mlp, feats, st,
                                            a.out_dim, lane);
        store_run(stage[wv], ro, j, n_k, a.out_dim, lane);
        wave_lds_sync();
    }
}

template <MlpKind K, int C>
hipError_t launch_batch_kind(const BatchArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s)
{
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        k_batch<K, H, NH, C><<<grid, kFrameThreads, 0, s>>>(a);                               \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

template <MlpKind K, int C, bool SH>
hipError_t launch_frame_kind(const FrameArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s)
{
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        k_frame<K, H, NH, C, SH><<<grid, kFrameThreads, 0, s>>>(a);                           \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

// per-precision entry points (frame_<precision>.hip)
hipError_t launch_frame_f32(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid, hipStream_t s);
hipError_t launch_frame_f16(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid, hipStream_t s);
hipError_t launch_frame_bf16(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid, hipStream_t s);
hipError_t launch_frame_fp8(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid, hipStream_t s);
hipError_t launch_frame_f32_mfma(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid,
                                 hipStream_t s);
hipError_t launch_calibrate_kernel(const FrameArgs &a, const MlpShape &sh, bool shared, unsigned grid,
                                   hipStream_t s);
hipError_t launch_batch_f16(const BatchArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s);
hipError_t launch_batch_f32(const BatchArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s);

}  // namespace bcf
