// The decoder MLP f_eta (eq. 3; ReLU hidden layers, linear output) on MFMA.
//
// One wave evaluates 16 queries per call. D = A * B + C with M = output
// units, N = the 16 queries, K = inputs. Lane L holds row L % 16 of A and the
// K slots of group g = L / 16 of B; the 16x16 D tile leaves rows 4g..4g+3 of
// query L % 16 in lane L, which becomes the next layer's B operand once the
// next layer's K slots are ordered to match (the host orders the weights):
//
//   P = 8 (16x16x32 f16 / bf16 / fp8): layer 0 slot (g, p): pyramid g, channel p (p < 3)
//                                      hidden slot (kc, g, p): unit 16 (2 kc + p / 4) + 4 g + p % 4
//   P = 1 (16x16x4 fp32):              layer 0 slot (kc, g): pyramid g, channel kc (kc < 3)
//                                      hidden slot (kc, g): unit 16 (kc / 4) + 4 g + kc % 4
//
// fp8 (OCP e4m3) stores weights scaled by a per-layer factor and quantises
// each layer's input with a static per-layer factor; the fp32 accumulator is
// rescaled before the bias.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace bcf {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr float kFp8Max = 448.0f;            // largest finite OCP e4m3 value

// max(x, 0) on the bit pattern: negative floats are negative integers. One
// integer max, without the NaN canonicalisation fmaxf needs.
__device__ __forceinline__ float relu(float x)
{
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int32_t, x), 0));
}

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Two fp32 values to a packed pair of f16 / bf16, rounded to nearest even:
// a two-element vector conversion, so that a pair always takes one
// instruction. (Not inline assembly: the compiler must see these reads of
// the MFMA results to put its wait states in front of them.)
__device__ __forceinline__ uint32_t cvt_pk_f16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2_t){a, b}, half2_t));
}
__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2_t){a, b}, bf16x2_t));
}

// max(x, 0) of both 16-bit floats (f16 or bf16) of a packed pair, again on
// the bit patterns: one packed integer max per two values
__device__ __forceinline__ uint32_t relu2(uint32_t w)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(short2_t, w), (short2_t){0, 0}));
}

// eight fp32 values to an f16 / bf16 operand, optionally after max(x, 0)
template <typename Op, bool BF16, bool RELU>
__device__ __forceinline__ Op pack16(const float *x)
{
    u32x4_t w;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t p = BF16 ? cvt_pk_bf16(x[2 * i], x[2 * i + 1]) : cvt_pk_f16(x[2 * i], x[2 * i + 1]);
        w[i] = RELU ? relu2(p) : p;
    }
    return __builtin_bit_cast(Op, w);
}

// The per-precision operand type. pack() converts 8 fp32 inputs (P = 8) or
// one (P = 1) to an operand; pack_relu() does the same for max(x, 0), the
// hidden layers' activation, in whichever order costs fewest instructions
// (rounding to f16, bf16 or fp8 commutes with max(., 0): both are monotonic
// and keep zero).
template <MlpKind K> struct Mma;

template <> struct Mma<MLP_MFMA_F16> {
    static constexpr int P = 8;
    static constexpr bool SCALED = false;
    typedef half8_t Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return *reinterpret_cast<const half8_t *>(p + 2 * e);
    }
    static __device__ __forceinline__ Op pack(const float *x, float) { return pack16<Op, false, false>(x); }
    static __device__ __forceinline__ Op pack_relu(const float *x, float) { return pack16<Op, false, true>(x); }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <> struct Mma<MLP_MFMA_BF16> {
    static constexpr int P = 8;
    static constexpr bool SCALED = false;
    typedef bf16x8_t Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return *reinterpret_cast<const bf16x8_t *>(p + 2 * e);
    }
    static __device__ __forceinline__ Op pack(const float *x, float) { return pack16<Op, true, false>(x); }
    static __device__ __forceinline__ Op pack_relu(const float *x, float) { return pack16<Op, true, true>(x); }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// lo = -kFp8Max: saturate to the finite e4m3 range; lo = 0: also max(x, 0)
template <bool RELU = false>
__device__ __forceinline__ uint32_t fp8x4(float a, float b, float c, float d)
{
    // saturate, then round to nearest even
    constexpr float lo = RELU ? 0.0f : -kFp8Max;
    a = __builtin_amdgcn_fmed3f(a, lo, kFp8Max);
    b = __builtin_amdgcn_fmed3f(b, lo, kFp8Max);
    c = __builtin_amdgcn_fmed3f(c, lo, kFp8Max);
    d = __builtin_amdgcn_fmed3f(d, lo, kFp8Max);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

template <> struct Mma<MLP_MFMA_FP8> {
    static constexpr int P = 8;
    static constexpr bool SCALED = true;
    typedef long Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return *reinterpret_cast<const long *>(p + e);
    }
    static __device__ __forceinline__ Op pack(const float *x, float inv_scale)
    {
        const uint32_t lo = fp8x4(x[0] * inv_scale, x[1] * inv_scale, x[2] * inv_scale, x[3] * inv_scale);
        const uint32_t hi = fp8x4(x[4] * inv_scale, x[5] * inv_scale, x[6] * inv_scale, x[7] * inv_scale);
        return (long)(((uint64_t)hi << 32) | lo);
    }
    // inv_scale > 0, so max(x, 0) * inv_scale = max(x * inv_scale, 0)
    static __device__ __forceinline__ Op pack_relu(const float *x, float inv_scale)
    {
        const uint32_t lo =
            fp8x4<true>(x[0] * inv_scale, x[1] * inv_scale, x[2] * inv_scale, x[3] * inv_scale);
        const uint32_t hi =
            fp8x4<true>(x[4] * inv_scale, x[5] * inv_scale, x[6] * inv_scale, x[7] * inv_scale);
        return (long)(((uint64_t)hi << 32) | lo);
    }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
    }
};

template <> struct Mma<MLP_MFMA_F32> {
    static constexpr int P = 1;
    static constexpr bool SCALED = false;
    typedef float Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return reinterpret_cast<const float *>(p)[e];
    }
    static __device__ __forceinline__ Op pack(const float *x, float) { return x[0]; }
    static __device__ __forceinline__ Op pack_relu(const float *x, float) { return relu(x[0]); }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// K chunks of a layer's input: layer 0 has 4 pyramids x 3 channels
template <int P> __host__ __device__ constexpr int kchunks0() { return P == 1 ? 3 : 1; }
template <int P> __host__ __device__ constexpr int kchunks_hidden(int H) { return P == 1 ? H / 4 : (H + 31) / 32; }

// MLP weights of one precision, held in registers for the whole kernel.
template <MlpKind K, int H, int NH>
struct MfmaMlp {
    typedef Mma<K> M;
    static constexpr int P = M::P;
    static constexpr int HB = H / 16;                   // M blocks of a hidden layer
    static constexpr int KC0 = kchunks0<P>();
    static constexpr int KCH = kchunks_hidden<P>(H);
    typename M::Op w0[HB][KC0], wh[NH > 1 ? NH - 1 : 1][HB][KCH], wo[KCH];
    float4_t b0[HB], bh[NH > 1 ? NH - 1 : 1][HB], bo;
    float deq[NH + 1], inv_in[NH + 1];                  // fp8 scales per layer

    __device__ __forceinline__ void load(const uint8_t *ws, const WsLayout &lay, uint32_t lane)
    {
        const uint32_t g = lane >> 4;
        const uint8_t *p = ws + lay.layer_w_off[0];
        const float *bb = reinterpret_cast<const float *>(ws + lay.layer_b_off[0]);
#pragma unroll
        for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) w0[mb][kc] = M::load(p, ((size_t)(mb * KC0 + kc) * 64 + lane) * P);
            b0[mb] = *reinterpret_cast<const float4_t *>(bb + 16 * mb + 4 * g);
        }
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            const uint8_t *ph = ws + lay.layer_w_off[l];
            const float *bh_ = reinterpret_cast<const float *>(ws + lay.layer_b_off[l]);
#pragma unroll
            for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
                for (int kc = 0; kc < KCH; ++kc)
                    wh[l - 1][mb][kc] = M::load(ph, ((size_t)(mb * KCH + kc) * 64 + lane) * P);
                bh[l - 1][mb] = *reinterpret_cast<const float4_t *>(bh_ + 16 * mb + 4 * g);
            }
        }
        const uint8_t *po = ws + lay.layer_w_off[NH];
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) wo[kc] = M::load(po, ((size_t)kc * 64 + lane) * P);
        bo = *reinterpret_cast<const float4_t *>(reinterpret_cast<const float *>(ws + lay.layer_b_off[NH]) + 4 * g);
        const float *sc = reinterpret_cast<const float *>(ws + lay.scales_off);
#pragma unroll
        for (int l = 0; l <= NH; ++l) {
            deq[l] = M::SCALED ? sc[2 * l] : 1.0f;
            inv_in[l] = M::SCALED ? sc[2 * l + 1] : 1.0f;
        }
    }

    // one layer: acc = W x (+ bias) for M block mb
    __device__ __forceinline__ float4_t finish(float4_t acc, float4_t bias, int l) const
    {
        if (M::SCALED) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = fmaf(acc[j], deq[l], bias[j]);
        }
        return acc;
    }

    // pack this lane's K slots of a hidden layer's output, after the ReLU, into chunk kc
    __device__ __forceinline__ typename M::Op hidden_chunk(const float (*act)[4], int kc, float inv) const
    {
        if (P == 1) return M::pack_relu(&act[kc / 4][kc % 4], inv);
        float x[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            x[j] = 2 * kc < HB ? act[2 * kc][j] : 0.0f;
            x[4 + j] = 2 * kc + 1 < HB ? act[2 * kc + 1][j] : 0.0f;
        }
        return M::pack_relu(x, inv);
    }

    // run() for G independent groups of 16 queries at once, layer by layer,
    // so that each layer's MFMAs of the different groups follow each other
    // and hide one another's latency
    template <int G>
    __device__ __forceinline__ void run_groups(const float (*f)[4], float4_t *out) const
    {
        const float4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
        typename M::Op x0[G][KC0];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (P == 1) {
#pragma unroll
                for (int kc = 0; kc < KC0; ++kc) x0[q][kc] = M::pack(f[q] + kc, 1.0f);
            } else {
                const float x[8] = {f[q][0], f[q][1], f[q][2], 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                x0[q][0] = M::pack(x, inv_in[0]);
            }
        }
        float act[G][HB][4];                           // pre-activations of the hidden layer
#pragma unroll
        for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                float4_t acc = M::SCALED ? zero : b0[mb];
#pragma unroll
                for (int kc = 0; kc < KC0; ++kc) acc = M::mma(w0[mb][kc], x0[q][kc], acc);
                acc = finish(acc, b0[mb], 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) act[q][mb][j] = acc[j];
            }
        }
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            typename M::Op xin[G][KCH];
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int kc = 0; kc < KCH; ++kc) xin[q][kc] = hidden_chunk(act[q], kc, inv_in[l]);
#pragma unroll
            for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    float4_t acc = M::SCALED ? zero : bh[l - 1][mb];
#pragma unroll
                    for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wh[l - 1][mb][kc], xin[q][kc], acc);
                    acc = finish(acc, bh[l - 1][mb], l);
#pragma unroll
                    for (int j = 0; j < 4; ++j) act[q][mb][j] = acc[j];
                }
            }
        }
        typename M::Op xin[G][KCH];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int kc = 0; kc < KCH; ++kc) xin[q][kc] = hidden_chunk(act[q], kc, inv_in[NH]);
#pragma unroll
        for (int q = 0; q < G; ++q) {
            float4_t acc = M::SCALED ? zero : bo;
#pragma unroll
            for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wo[kc], xin[q][kc], acc);
            out[q] = finish(acc, bo, NH);
        }
    }

    // f: this lane's layer-0 inputs (pyramid g = lane / 16, channels 0..2, 0)
    // of query lane % 16; returns output rows 4g..4g+3 of that query
    __device__ __forceinline__ float4_t run(const float f[4]) const
    {
        const float4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
        typename M::Op x0[KC0];
        if (P == 1) {
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) x0[kc] = M::pack(f + kc, 1.0f);
        } else {
            const float x[8] = {f[0], f[1], f[2], 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            x0[0] = M::pack(x, inv_in[0]);
        }
        float act[HB][4];                               // pre-activations of the hidden layer
#pragma unroll
        for (int mb = 0; mb < HB; ++mb) {
            float4_t acc = M::SCALED ? zero : b0[mb];
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) acc = M::mma(w0[mb][kc], x0[kc], acc);
            acc = finish(acc, b0[mb], 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) act[mb][j] = acc[j];
        }
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            typename M::Op xin[KCH];
#pragma unroll
            for (int kc = 0; kc < KCH; ++kc) xin[kc] = hidden_chunk(act, kc, inv_in[l]);
#pragma unroll
            for (int mb = 0; mb < HB; ++mb) {
                float4_t acc = M::SCALED ? zero : bh[l - 1][mb];
#pragma unroll
                for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wh[l - 1][mb][kc], xin[kc], acc);
                acc = finish(acc, bh[l - 1][mb], l);
#pragma unroll
                for (int j = 0; j < 4; ++j) act[mb][j] = acc[j];
            }
        }
        typename M::Op xin[KCH];
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) xin[kc] = hidden_chunk(act, kc, inv_in[NH]);
        float4_t acc = M::SCALED ? zero : bo;
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wo[kc], xin[kc], acc);
        return finish(acc, bo, NH);
    }
};

}  // namespace bcf
