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

template <int H, int NH, int C>
__device__ __forceinline__ void mlp_valu(const FrameArgs &a, const float z[12], float o[C], float *amax)
{
    const_float *W = constant_floats(a.ws + a.lay.layer_w_off[0]);
    const_float *B = constant_floats(a.ws + a.lay.layer_b_off[0]);
    if (amax) {
#pragma unroll
        for (int i = 0; i < 12; ++i) amax[0] = fmaxf(amax[0], fabsf(z[i]));
    }
    float hcur[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float acc = B[j];
#pragma unroll
        for (int i = 0; i < 12; ++i) acc = fmaf(W[j * 12 + i], z[i], acc);
        hcur[j] = relu(acc);
    }
#pragma unroll
    for (int l = 1; l < NH; ++l) {
        if (amax) {
#pragma unroll
            for (int i = 0; i < H; ++i) amax[l] = fmaxf(amax[l], hcur[i]);
        }
        W = constant_floats(a.ws + a.lay.layer_w_off[l]);
        B = constant_floats(a.ws + a.lay.layer_b_off[l]);
        float hn[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float acc = B[j];
#pragma unroll
            for (int i = 0; i < H; ++i) acc = fmaf(W[j * H + i], hcur[i], acc);
            hn[j] = relu(acc);
        }
#pragma unroll
        for (int j = 0; j < H; ++j) hcur[j] = hn[j];
    }
    if (amax) {
#pragma unroll
        for (int i = 0; i < H; ++i) amax[NH] = fmaxf(amax[NH], hcur[i]);
    }
    W = constant_floats(a.ws + a.lay.layer_w_off[NH]);
    B = constant_floats(a.ws + a.lay.layer_b_off[NH]);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        float acc = B[j];
#pragma unroll
        for (int i = 0; i < H; ++i) acc = fmaf(W[j * H + i], hcur[i], acc);
        o[j] = acc;
    }
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

template <MlpKind K, int H, int NH, int C, bool SHARED>
__global__ void __launch_bounds__(kFrameThreads) k_frame(FrameArgs a)
{
    constexpr bool VALU = K == MLP_VALU_F32;
    __shared__ LevelLut lut;
    __shared__ float4_t feats[VALU ? 1 : kFrameWaves][64][4];
    __shared__ float4_t stage[kFrameWaves][64 * kMaxOut / 4];
    copy_lut(a.lut, lut);

    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ws + a.lay.scratch_off, (uint32_t)a.lay.scratch_bytes);
    const __amdgpu_buffer_rsrc_t rq = make_rsrc(a.queries, a.n * 12u);
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out, a.n * a.out_dim * 4u);
    MfmaMlp<VALU ? MLP_MFMA_F16 : K, H, NH> mlp;
    if (!VALU) mlp.load(a.ws, a.lay, lane);
    float *st = reinterpret_cast<float *>(&stage[wv][0]);
    const uint32_t g = lane >> 4, qi = lane & 15;

    const uint32_t n_iter = (a.n + 63) / 64;
    const uint32_t n_waves = gridDim.x * kFrameWaves;
    for (uint32_t it = blockIdx.x * kFrameWaves + wv; it < n_iter; it += n_waves) {
        const uint32_t q = it * 64 + lane;
        // queries past n read as zeros (buffer range check); their rows are not stored
        const Query qq = load_query(rq, q);
        float z[12];
        filter4<SHARED>(rs, lut, a.levels_bias, a.stride, qq.u, qq.v, qq.s, z);
        if (VALU) {
            float o[C];
            mlp_valu<H, NH, C>(a, z, o, nullptr);
#pragma unroll
            for (int j = 0; j < C; ++j)
                if ((uint32_t)j < a.out_dim) st[lane * a.out_dim + j] = o[j];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float4_t v4 = {z[3 * t], z[3 * t + 1], z[3 * t + 2], 0.0f};
                feats[wv][lane][t] = v4;
            }
            wave_lds_sync();
#pragma unroll
            for (int grp = 0; grp < 4; ++grp) {
                const float4_t f4 = feats[wv][16 * grp + qi][g];
                const float f[4] = {f4[0], f4[1], f4[2], f4[3]};
                const float4_t o4 = mlp.run(f);
                const uint32_t row = (16 * grp + qi) * a.out_dim;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (4 * g + j < a.out_dim) st[row + 4 * g + j] = o4[j];
            }
        }
        wave_lds_sync();
        // the wave's rows are 64 * out_dim contiguous floats (a multiple of 16 bytes)
        const uint32_t base = it * 64u * a.out_dim * 4u;
        if (it * 64 + 64 <= a.n) {
            const uint32_t chunks = 16 * a.out_dim;
            for (uint32_t k = lane; k < chunks; k += 64)
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4_t, stage[wv][k]), ro,
                                                       (int)(base + 16u * k), 0, 0);
        } else {                                       // last, partial iteration
            const uint32_t floats = (a.n - it * 64) * a.out_dim;
            for (uint32_t k = lane; k < floats; k += 64)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, st[k]), ro,
                                                      (int)(base + 4u * k), 0, 0);
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
        mlp_valu<H, NH, C>(a, z, o, amax);
    }
#pragma unroll
    for (int l = 0; l <= NH; ++l) {
        // non-negative floats order like their bit patterns
        atomicMax(reinterpret_cast<unsigned int *>(a.absmax) + l, __builtin_bit_cast(unsigned int, amax[l]));
    }
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

}  // namespace bcf
