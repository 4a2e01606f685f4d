// The decode and calibration kernels, instantiated per MLP precision in
// frame_<precision>.hip (separate translation units compile in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

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
// Outputs are staged in LDS so each wave writes its 64 rows with coalesced
// buffer stores.

constexpr int kFrameThreads = 256;
constexpr int kFrameWaves = kFrameThreads / 64;
// a wave's 64 feature vectors (4 x float4 each) fit its output stage
static_assert(64 * 4 <= 64 * kMaxOut / 4, "feature vectors must fit the output stage");

// Cache policy of the output stores: non-temporal (streamed). The kernels
// never read their outputs back; on the frame benchmark the decode runs about
// a quarter faster with its output stream marked so.
constexpr int kStoreNT = 2;   // the buffer intrinsics' cache-policy bit for "nt"

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
    // a wave takes a tile of kTileW columns by kTileH rows (lane = row *
    // kTileW + column); with 0, 64 consecutive queries.
    // wide: every output row this launch writes starts on a 16-byte boundary
    // and n * out_dim is a multiple of 4, so items store 16-byte chunks
    uint32_t grid_w, tiles_x, n_items, wide;
    // tiled work: tiles_y rows of tiles; strip_rows > 0: the tile rows form
    // strips of that many, dealt to the XCDs in turn (0: items round-robin).
    // Linear work is laid out the same way, as rows of tiles_x items.
    uint32_t tiles_y, strip_rows;
};

// Work-item tiles for queries declared as an image: 16 x 4.
constexpr uint32_t kTileLog2 = 4, kTileW = 1u << kTileLog2, kTileH = 64u >> kTileLog2;

// The grid is a multiple of the 8 XCDs, to which workgroups are dispatched
// round-robin (workgroup b runs on XCD b % 8), and a small multiple of what
// is resident at once, so the waves sweep the image nearly together. Tiled
// work deals strips of whole tile rows to the XCDs in turn (strip j to XCD
// j % 8); an XCD's waves walk its strips tile by tile. Texels are shared
// along a strip -- a textured plane that wraps repeats the same texels
// across the image's width -- so whole-width strips keep that sharing inside
// one XCD's L2, while the strips of different XCDs share only their edge
// rows. Linear work is dealt the same way in runs of kLinearRun items
// (consecutive queries share texels along a scanline); images or runs too
// few to give every XCD one go round-robin over all waves.
constexpr uint32_t kXcds = 8;
constexpr uint32_t kLinearRun = 64;     // 64-query items per run of linear work dealt to one XCD

// A wave's share of the work: items first, first + step, ... below end. In
// strip mode item k is tile k % per of strip (k / per) * kXcds + xcd, per =
// strip_rows * tiles_x tiles; otherwise item k is tile k (row-major).
struct WaveWork {
    uint32_t first, end, step, xcd, per;
};

__device__ __forceinline__ WaveWork wave_work(const FrameArgs &a, uint32_t wv)
{
    if (a.strip_rows) {
        const uint32_t x = blockIdx.x % kXcds;
        const uint32_t n_strips = (a.tiles_y + a.strip_rows - 1) / a.strip_rows;
        const uint32_t mine = n_strips > x ? (n_strips - x + kXcds - 1) / kXcds : 0;   // strips x, x + 8, ...
        const uint32_t per = a.strip_rows * a.tiles_x;
        return WaveWork{(blockIdx.x / kXcds) * kFrameWaves + wv, mine * per, (gridDim.x / kXcds) * kFrameWaves, x,
                        per};
    }
    return WaveWork{blockIdx.x * kFrameWaves + wv, a.n_items, gridDim.x * kFrameWaves, 0, 0};
}

struct ItemRange {
    uint32_t first, end, step;
};

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
        // lane (g, qi) holds outputs 4g .. 4g + 3 of its query; those past
        // out_dim go to the stage's last float, which 64 rows of fewer than
        // kMaxOut outputs never use (a select, not a branch per output)
        constexpr uint32_t kSpare = 64 * kMaxOut - 1;
        float f[4][4];
#pragma unroll
        for (int grp = 0; grp < 4; ++grp)
#pragma unroll
            for (int i = 0; i < 4; ++i) f[grp][i] = fin[grp][i];
        float4_t o[4];
        mlp.template run_groups<4>(f, o);
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            const float4_t o4 = o[grp];
            const uint32_t row = (16 * grp + qi) * out_dim;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                st[4 * g + j < out_dim ? row + 4 * g + j : kSpare] = o4[j];
        }
    }
    wave_lds_sync();
}

// One wave's 64 queries: filter (eqs. 9, 10), concatenate, MLP.
template <MlpKind K, int H, int NH, int C, int LAYOUT>
__device__ __forceinline__ void decode_wave(const Query &qq, __amdgpu_buffer_rsrc_t rs, const LevelLut &lut,
                                            const float *levels_bias, uint32_t stride, const uint8_t *wbase,
                                            const WsLayout &lay,
                                            const MfmaMlp<K == MLP_VALU_F32 ? MLP_MFMA_F16 : K, H, NH> &mlp,
                                            float4_t (*feats)[4], float *st, uint32_t out_dim, uint32_t lane)
{
    float z[12];
    filter4<LAYOUT>(rs, lut, levels_bias, stride, qq.u, qq.v, qq.s, z);
    mlp_stage<K, H, NH, C>(z, wbase, lay, mlp, feats, st, out_dim, lane);
}

// decode_wave for a material with a position-interleaved scratch
template <MlpKind K, int H, int NH, int C>
__device__ __forceinline__ void decode_wave_interleaved(const Query &qq, __amdgpu_buffer_rsrc_t rs,
                                                        const LevelLut &lut, const float *levels_bias,
                                                        const uint8_t *wbase, const WsLayout &lay,
                                                        const MfmaMlp<K == MLP_VALU_F32 ? MLP_MFMA_F16 : K, H, NH> &mlp,
                                                        float4_t (*feats)[4], float *st, uint32_t out_dim,
                                                        uint32_t lane)
{
    PendingPacked taps;
    fetch4_packed(rs, lut, levels_bias, qq.u, qq.v, qq.s, taps);
    float z[12];
    filter_pending_packed(taps, z);
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
                                                   0, kStoreNT);
    } else {
        const float *st = reinterpret_cast<const float *>(stage);
        const uint32_t floats = (n - it * 64) * out_dim;
        for (uint32_t k = lane; k < floats; k += 64)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, st[k]), ro, (int)(base + 4u * k), 0,
                                                  kStoreNT);
    }
}

// Stores of one work item: always 16 / V buffer stores of V floats per lane
// (V = 4 when FrameArgs::wide, else 1) and no branches around them. An item's
// output is a set of runs of contiguous floats: one run of 64 * out_dim for
// linear items, one of kTileW * out_dim per tile row for tiled items. The
// lanes of a run take its V-float chunks in turn; a chunk with nowhere to go
// (past the run, the image's right edge or the output's end) is sent to
// `oob`, the first byte past the output buffer, which the buffer range check
// drops. Stores count in the same in-order counter as loads; a fixed count
// lets the compiler wait for a load issued before these stores without
// waiting for the stores themselves.
template <int V>
__device__ __forceinline__ void store_item(const FrameArgs &a, uint32_t oob, const float *st,
                                           __amdgpu_buffer_rsrc_t ro, uint32_t it, uint32_t row0, uint32_t col0,
                                           uint32_t lane)
{
    typedef float vec_t __attribute__((ext_vector_type(V)));
    const uint32_t n_out = a.n * a.out_dim;
    uint32_t e0, step, k0, base, lim;
    if (!a.grid_w) {
        base = it * 64u * a.out_dim;
        lim = min(64u * a.out_dim, n_out - min(base, n_out));
        e0 = V * lane;
        step = 64u * V;
        k0 = 0;
    } else {
        const uint32_t r = lane >> kTileLog2;
        base = ((row0 + r) * a.grid_w + col0) * a.out_dim;
        lim = min(kTileW, a.grid_w - col0) * a.out_dim;
        lim = min(lim, n_out - min(base, n_out));
        e0 = V * (lane & (kTileW - 1u));
        step = kTileW * V;
        k0 = r * kTileW * a.out_dim;
    }
#pragma unroll
    for (int m = 0; m < 16 / V; ++m) {
        const uint32_t e = e0 + step * m;
        const vec_t v = *reinterpret_cast<const vec_t *>(st + k0 + e);
        const int off = (int)(e < lim ? (base + e) * 4u : oob);
        if constexpr (V == 4)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4_t, v), ro, off, 0, kStoreNT);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), ro, off, 0, kStoreNT);
    }
}

// 16 / V stores past the output's end: the loop's entry then has the same
// stores outstanding as its back edge.
template <int V>
__device__ __forceinline__ void store_dummies(__amdgpu_buffer_rsrc_t ro, uint32_t oob)
{
#pragma unroll
    for (int m = 0; m < 16 / V; ++m) {
        uint32_t o = oob;
        asm volatile("" : "+v"(o));           // separate stores, not merged into wider ones
        if constexpr (V == 4)
            __builtin_amdgcn_raw_buffer_store_b128(uint4_t{0, 0, 0, 0}, ro, (int)o, 0, kStoreNT);
        else
            __builtin_amdgcn_raw_buffer_store_b32(0u, ro, (int)o, 0, kStoreNT);
    }
}

template <int V>
struct Width {
    static constexpr int value = V;
};

template <MlpKind K, int H, int NH, int C, int LAYOUT>
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

    const uint32_t oob = a.n * a.out_dim * 4u;
    const WaveWork w = wave_work(a, wv);
    if (w.first >= w.end) return;
    // Item k of this wave's share: sets `it` (the linear item, or the tile
    // row) and the tile's origin, and returns this lane's query; lanes outside
    // the image or past n (also whole tiles of a strip below the image) read
    // zeros (buffer range check) and their rows are not stored.
    auto query_of = [&](uint32_t k, uint32_t &it, uint32_t &row0, uint32_t &col0) -> uint32_t {
        uint32_t tr, tc;
        if (w.per) {
            const uint32_t j = k / w.per, rem = k - j * w.per;
            tr = (j * kXcds + w.xcd) * a.strip_rows + rem / a.tiles_x;
            tc = rem % a.tiles_x;
        } else {
            tr = k / a.tiles_x;
            tc = k - tr * a.tiles_x;
        }
        if (!a.grid_w) {                  // linear work: rows of tiles_x items
            it = tr * a.tiles_x + tc;
            row0 = col0 = 0;
            return it * 64 + lane;
        }
        it = tr;
        row0 = tr * kTileH;
        col0 = tc * kTileW;
        const uint32_t col = col0 + (lane & (kTileW - 1u));
        const uint32_t q = (row0 + (lane >> kTileLog2)) * a.grid_w + col;
        return col < a.grid_w && q < a.n ? q : a.n;
    };
    const ItemRange items{w.first, w.end, w.step};
    auto run = [&](auto width) {
        constexpr int V = decltype(width)::value;
        uint32_t it, row0, col0, i_, r_, c_;
        if (LAYOUT != kLayoutSplit) {
            // Per item: blend its texels, run the MLP, issue the next item's
            // texel loads and the query after that, then store -- so the
            // wait for the next texels never includes these stores. The loop
            // is entered the way it repeats (texel loads, a query load, the
            // stores), and the last item fetches its first item again, so
            // every path into the loop's top has the same loads and stores
            // outstanding.
            using Taps = std::conditional_t<LAYOUT == kLayoutPacked, PendingPacked, PendingTaps>;
            auto fetch = [&](const Query &q, Taps &t) {
                if constexpr (LAYOUT == kLayoutPacked) fetch4_packed(rs, lut, a.levels_bias, q.u, q.v, q.s, t);
                else fetch4_shared(rs, lut, a.levels_bias, a.stride, q.u, q.v, q.s, t);
            };
            auto clamp_item = [&](uint32_t k) { return k < items.end ? k : items.first; };
            const Query q0 = load_query(rq, query_of(items.first, i_, r_, c_));
            Taps taps;
            fetch(q0, taps);
            Query qnext = load_query(rq, query_of(clamp_item(items.first + items.step), i_, r_, c_));
            store_dummies<V>(ro, oob);
            for (uint32_t k = items.first; k < items.end; k += items.step) {
                query_of(k, it, row0, col0);
                float z[12];
                if constexpr (LAYOUT == kLayoutPacked) filter_pending_packed(taps, z);
                else filter_pending(taps, z);
                mlp_stage<K, H, NH, C>(z, a.ws, a.lay, mlp, feats, st, a.out_dim, lane);
                fetch(qnext, taps);
                qnext = load_query(rq, query_of(clamp_item(k + 2 * items.step), i_, r_, c_));
                store_item<V>(a, oob, st, ro, it, row0, col0, lane);
                wave_lds_sync();
            }
        } else {
            // the next item's query is loaded while this item's texels are fetched
            Query next = load_query(rq, query_of(items.first, i_, r_, c_));
            for (uint32_t k = items.first; k < items.end; k += items.step) {
                query_of(k, it, row0, col0);
                const Query qq = next;
                if (k + items.step < items.end) next = load_query(rq, query_of(k + items.step, i_, r_, c_));
                decode_wave<K, H, NH, C, kLayoutSplit>(qq, rs, lut, a.levels_bias, a.stride, a.ws, a.lay, mlp, feats,
                                                 st, a.out_dim, lane);
                store_item<V>(a, oob, st, ro, it, row0, col0, lane);
                wave_lds_sync();
            }
        }
    };
    if (a.wide)
        run(Width<4>());
    else
        run(Width<1>());
}

// The plain fp32 decode that records each layer's largest input magnitude
// (the static fp8 activation scales come from a calibration batch).
template <int H, int NH, int C, int LAYOUT>
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
        filter4<LAYOUT>(rs, lut, a.levels_bias, a.stride, qq.u, qq.v, qq.s, z);
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
    uint32_t scratch_bytes, stride, shared, interleaved;   // interleaved: as MaterialDesc
    uint32_t seg_chunk[kMaxLevels];        // interleaved: first unpack chunk of each level's segment
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
    uint32_t interleave;                   // 1: waves interleave runs of items; 0: contiguous ranges
    uint32_t run;                          // interleaved: consecutive items (of 64 queries) a wave takes
};

// Query range of material k: the caller's offsets clamped to [0, n_total],
// made non-decreasing, at most kMaxQueriesPerLaunch queries.
__device__ __forceinline__ void batch_range(const BatchArgs &a, uint32_t k, uint32_t &q0, uint32_t &cnt)
{
    q0 = min(a.offsets[k], a.n_total);
    const uint32_t q1 = max(min(a.offsets[k + 1], a.n_total), q0);
    cnt = min(q1 - q0, (uint32_t)kMaxQueriesPerLaunch);
}

// W waves per workgroup (the autotuner picks 2 or 4).
template <MlpKind K, int H, int NH, int C, int W>
__global__ void __launch_bounds__(64 * W) k_batch(BatchArgs a)
{
    constexpr bool VALU = K == MLP_VALU_F32;
    __shared__ LevelLut lut[W];                           // each wave's current material
    __shared__ float4_t stage[W][64 * kMaxOut / 4];       // features, then output rows
    // the wave index is uniform across the wave: say so, so that everything
    // derived from it (work items, materials, offsets) lives in SGPRs
    const uint32_t lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *st = reinterpret_cast<float *>(&stage[wv][0]);
    float4_t (*feats)[4] = reinterpret_cast<float4_t (*)[4]>(&stage[wv][0]);
    const uint32_t total = a.items[a.n_mats];

    // interleaved: wave g takes runs of `run` consecutive items, g-th run of
    // every gridDim.x * W; contiguous: the XCD's band split into one range per wave
    ItemRange items;
    uint32_t run = 1;
    if (a.interleave) {
        run = max(a.run, 1u);
        items = ItemRange{(blockIdx.x * W + wv) * run, total, gridDim.x * W * run};
    } else {
        const uint32_t xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds;
        const uint32_t waves = (gridDim.x / kXcds) * W, w = local * W + wv;
        const uint64_t lo = (uint64_t)total * xcd / kXcds, hi = (uint64_t)total * (xcd + 1) / kXcds;
        items.first = (uint32_t)(lo + (hi - lo) * w / waves);
        items.end = (uint32_t)(lo + (hi - lo) * (w + 1) / waves);
        items.step = 1;
    }

    MfmaMlp<VALU ? MLP_MFMA_F16 : K, H, NH> mlp;
    uint32_t cur = 0xFFFFFFFFu, first_item = 0, n_k = 0, shared = 0, interleaved = 0, stride = 0;
    float lb[2 * kMaxTextures];
    const uint8_t *wbase = a.ws;
    __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ws, 0), rq = rs, ro = rs;
    for (uint32_t it0 = items.first; it0 < items.end; it0 += items.step)
    for (uint32_t it = it0; it < min(it0 + run, items.end); ++it) {
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
            interleaved = uniform(M.interleaved);
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
        if (interleaved)
            decode_wave_interleaved<K, H, NH, C>(qq, rs, lut[wv], lb, wbase, a.lay, mlp, feats, st, a.out_dim,
                                                 lane);
        else if (shared)
            decode_wave<K, H, NH, C, kLayoutShared>(qq, rs, lut[wv], lb, stride, wbase, a.lay, mlp, feats, st,
                                           a.out_dim, lane);
        else
            decode_wave<K, H, NH, C, kLayoutSplit>(qq, rs, lut[wv], lb, stride, wbase, a.lay, mlp, feats, st,
                                            a.out_dim, lane);
        store_run(stage[wv], ro, j, n_k, a.out_dim, lane);
        wave_lds_sync();
    }
}

template <MlpKind K, int C>
hipError_t launch_batch_kind(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s)
{
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        if (waves == 2) k_batch<K, H, NH, C, 2><<<grid, 128, 0, s>>>(a);                      \
        else k_batch<K, H, NH, C, 4><<<grid, 256, 0, s>>>(a);                                 \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

// Workgroups of KERNEL resident at once on the current device, 0 if the
// runtime cannot say (cached per kernel and device; concurrent first calls
// compute the same value).
template <auto KERNEL>
unsigned resident_workgroups()
{
    static std::atomic<int> cache[16];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    if (dev < 16) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return (unsigned)c;
    }
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, KERNEL, kFrameThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int r = std::max(per_cu, 1) * std::max(cus, 1);
    if (dev < 16) cache[dev].store(r, std::memory_order_relaxed);
    return (unsigned)r;
}

// One workgroup per kFrameWaves items, at most `cap`, a multiple of the XCDs.
// The cap is a small multiple of the workgroups resident at once: twice for
// the MFMA kernels, four times for the fp32 vector-ALU kernel (measured on
// the frame benchmark: the MFMA kernels run fastest when their waves sweep
// the image nearly together, the ALU-bound one with more waves queued behind
// the resident ones to fill the tail).
inline unsigned frame_launch_grid(uint32_t n_items, unsigned cap)
{
    const unsigned want = (n_items + kFrameWaves - 1) / kFrameWaves;
    cap = std::max(kXcds, cap / kXcds * kXcds);
    return std::min(std::max(kXcds, (want + kXcds - 1) / kXcds * kXcds), cap);
}

template <MlpKind K, int C, int SH>
hipError_t launch_frame_kind(const FrameArgs &a, const MlpShape &sh, hipStream_t s)
{
    constexpr unsigned kOversub = K == MLP_VALU_F32 ? 4 : 2;
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        const unsigned res = resident_workgroups<k_frame<K, H, NH, C, SH>>();                \
        k_frame<K, H, NH, C, SH>                                                              \
            <<<frame_launch_grid(a.n_items, res ? kOversub * res : 4096u), kFrameThreads, 0, s>>>(a); \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

// per-precision entry points (frame_<precision>.hip)
// layout: kLayoutSplit, kLayoutShared or kLayoutPacked (filter_device.hpp)
hipError_t launch_frame_f32(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s);
hipError_t launch_frame_f16(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s);
hipError_t launch_frame_bf16(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s);
hipError_t launch_frame_fp8(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s);
hipError_t launch_frame_f32_mfma(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s);
hipError_t launch_calibrate_kernel(const FrameArgs &a, const MlpShape &sh, int layout, unsigned grid,
                                   hipStream_t s);
hipError_t launch_batch_f16(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s);
hipError_t launch_batch_f32(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s);

}  // namespace bcf
