// Decode kernels for gfx950 (MI355X).
//
//  k_decode_blocks   BC6H blocks -> half bit patterns, one lane per block
//  k_predecode       every block of every pyramid -> texel scratch (r,g,b,0 halves)
//  k_prepare         MLP parameters -> padded per-precision operand layout
//  k_filter_mlp_*    per query: trilinear filter of every pyramid from the texel
//                    scratch (eq. 9 at s_i = s + b_i, eq. 10), concatenation, and
//                    the decoder MLP (eq. 3) on the vector ALU or on MFMA
#include <hip/hip_runtime.h>

#include "bc6h_device.hpp"
#include "internal.hpp"

namespace bcf {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ void load_table(uint32_t *lds)
{
    for (int i = threadIdx.x; i < kTableWords; i += blockDim.x) lds[i] = kTable[i];
    __syncthreads();
}

__device__ __forceinline__ float half_bits_to_float(uint32_t bits)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
}

__device__ __forceinline__ uint16_t float_to_bf16_rne(float x)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// blocks -> halves

template <bool SIGNED>
__global__ void __launch_bounds__(256) k_decode_blocks(const uint4 *__restrict__ blocks, size_t n,
                                                       uint16_t *__restrict__ out)
{
    __shared__ uint32_t table[kTableWords];
    load_table(table);
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 b = blocks[i];
    Bc6hHeader h;
    bc6h_header<SIGNED>(b.x, b.y, b.z, b.w, table, h);
    uint32_t packed[24];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int k = 3 * t + c;
            const uint32_t v = bc6h_texel<SIGNED>(h, (uint32_t)t, c);
            if (k & 1) packed[k >> 1] |= v << 16;
            else packed[k >> 1] = v;
        }
    }
    uint4 *dst = reinterpret_cast<uint4 *>(out + 48 * i);
#pragma unroll
    for (int j = 0; j < 6; ++j)
        dst[j] = make_uint4(packed[4 * j], packed[4 * j + 1], packed[4 * j + 2], packed[4 * j + 3]);
}

hipError_t launch_decode_blocks(const uint4 *blocks, size_t n, uint32_t is_signed, uint16_t *out,
                                hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (is_signed) k_decode_blocks<true><<<grid, 256, 0, s>>>(blocks, n, out);
    else k_decode_blocks<false><<<grid, 256, 0, s>>>(blocks, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// every block -> texel scratch. Level l of texture t is a row-major array of
// max(w>>l,1) x max(h>>l,1) texels of 8 bytes (r | g << 16, b) starting at
// texel tex_off[l].

struct PredecodeArgs {
    MaterialDesc m;
    PredecodePlan p;
    uint2 *texels;
};

template <bool SIGNED>
__global__ void __launch_bounds__(256) k_predecode(PredecodeArgs a)
{
    __shared__ uint32_t table[kTableWords];
    load_table(table);
    // segment of this workgroup (uniform scan over at most 64 entries)
    const uint32_t wg = blockIdx.x;
    uint32_t seg = 0;
    while (seg + 1 < a.p.n_seg && a.p.seg_wg[seg + 1] <= wg) ++seg;
    const TexDesc &T = a.m.tex[a.p.seg_tex[seg]];
    const uint32_t l = a.p.seg_lvl[seg];
    const uint32_t lw = max(T.w >> l, 1u), lh = max(T.h >> l, 1u);
    const uint32_t bx = (lw + 3) / 4, by = (lh + 3) / 4;
    const uint32_t bi = (wg - a.p.seg_wg[seg]) * 256 + threadIdx.x;
    if (bi >= bx * by) return;
    const uint4 b = T.blocks[T.blk_off[l] + bi];
    Bc6hHeader h;
    bc6h_header<SIGNED>(b.x, b.y, b.z, b.w, table, h);
    const uint32_t x0 = 4 * (bi % bx), y0 = 4 * (bi / bx);
    uint2 *dst = a.texels + T.tex_off[l];
    // A level narrower or shorter than 4 texels keeps only the top-left part
    // of its blocks in that direction.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (y0 + r >= lh) break;
        uint2 px[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t t = 4 * r + c;
            px[c].x = bc6h_texel<SIGNED>(h, t, 0) | bc6h_texel<SIGNED>(h, t, 1) << 16;
            px[c].y = bc6h_texel<SIGNED>(h, t, 2);
        }
        uint2 *row = dst + (size_t)(y0 + r) * lw + x0;
        if (lw >= 4) {        // x0 and the level's row starts are multiples of 4 texels (32 B)
            reinterpret_cast<uint4 *>(row)[0] = make_uint4(px[0].x, px[0].y, px[1].x, px[1].y);
            reinterpret_cast<uint4 *>(row)[1] = make_uint4(px[2].x, px[2].y, px[3].x, px[3].y);
        } else {
#pragma unroll
            for (uint32_t c = 0; c < 4; ++c)
                if (c < lw) row[c] = px[c];
        }
    }
}

hipError_t launch_predecode(const MaterialDesc &m, const PredecodePlan &p, uint2 *texels, hipStream_t s)
{
    PredecodeArgs a{m, p, texels};
    const unsigned grid = p.seg_wg[p.n_seg];
    if (grid == 0) return hipSuccess;
    if (m.is_signed) k_predecode<true><<<grid, 256, 0, s>>>(a);
    else k_predecode<false><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MLP operand layouts
//
// VALU: layer l is W[rows][cols] fp32 row-major then b[rows], rows/cols padded
// (layer 0 cols = 12: z0 index 3*texture + channel).
//
// MFMA 16x16xK (D = A * B + C, M = output units, N = 16 queries, K = inputs).
// Lane L holds A row m = L % 16 and P consecutive K slots of group g = L / 16;
// the 16x16 D tile leaves rows 4g..4g+3 in lane L, which is exactly the B
// operand layout of the next layer once the K slots are ordered to match.
// Storage per layer: [mblock][kchunk][lane][P] elements. K slot (kc, g, p):
//   P = 4 (fp16/bf16, 16x16x16):  layer 0: texture g, channel p (p < 3)
//                                  hidden:  unit 16 kc + 4 g + p
//   P = 1 (fp32, 16x16x4):         layer 0: texture g, channel kc (kc < 3)
//                                  hidden:  unit 16 (kc / 4) + 4 g + kc % 4
// The bias stays fp32 in natural order, padded to the M blocks.

__host__ __device__ inline uint32_t mfma_p(MlpKind k) { return k == MLP_MFMA_F32 ? 1u : 4u; }

__host__ __device__ inline uint32_t layer_in(const MlpShape &s, uint32_t l)
{
    return l == 0 ? 12u : s.hidden;
}

__host__ __device__ inline uint32_t layer_out(const MlpShape &s, uint32_t l, MlpKind k)
{
    if (l < s.n_hidden) return s.hidden;
    return k == MLP_VALU_F32 ? (s.out <= 10 ? 10u : 16u) : 16u;
}

__host__ __device__ inline uint32_t layer_kchunks(const MlpShape &s, uint32_t l, MlpKind k)
{
    if (k == MLP_MFMA_F32) return l == 0 ? 3u : s.hidden / 4;
    return l == 0 ? 1u : s.hidden / 16;
}

// logical input unit of K slot (kc, g, p) of layer l, or -1 for padding
__host__ __device__ inline int mfma_in_unit(const MlpShape &s, uint32_t l, MlpKind k, uint32_t kc,
                                            uint32_t g, uint32_t p)
{
    if (k == MLP_MFMA_F32) {
        if (l == 0) return (kc < 3) ? (int)(3 * g + kc) : -1;
        return (int)(16 * (kc / 4) + 4 * g + kc % 4);
    }
    if (l == 0) return p < 3 ? (int)(3 * g + p) : -1;
    return (int)(16 * kc + 4 * g + p);
}

__host__ __device__ inline size_t layer_elems(const MlpShape &s, uint32_t l, MlpKind k)
{
    if (k == MLP_VALU_F32) return (size_t)layer_out(s, l, k) * layer_in(s, l);
    return (size_t)(layer_out(s, l, k) / 16) * layer_kchunks(s, l, k) * 64 * mfma_p(k);
}

struct PrepareArgs {
    const float *params;
    MlpShape sh;
    MlpKind kind;
    WsLayout lay;
    uint8_t *ws;
};

// true-layout parameter W_l[o][i] (0 outside the true shape)
__device__ inline float param_w(const PrepareArgs &a, uint32_t l, int o, int i)
{
    size_t off = 0;
    for (uint32_t j = 0; j < l; ++j) off += (size_t)a.sh.dims[j] * a.sh.dims[j + 1] + a.sh.dims[j + 1];
    const uint32_t n_in = a.sh.dims[l], n_out = a.sh.dims[l + 1];
    if (o < 0 || i < 0 || (uint32_t)o >= n_out || (uint32_t)i >= n_in) return 0.0f;
    return a.params[off + (size_t)o * n_in + i];
}

__device__ inline float param_b(const PrepareArgs &a, uint32_t l, uint32_t o)
{
    size_t off = 0;
    for (uint32_t j = 0; j < l; ++j) off += (size_t)a.sh.dims[j] * a.sh.dims[j + 1] + a.sh.dims[j + 1];
    const uint32_t n_in = a.sh.dims[l], n_out = a.sh.dims[l + 1];
    return o < n_out ? a.params[off + (size_t)n_in * n_out + o] : 0.0f;
}

__global__ void k_prepare(PrepareArgs a)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t L = a.sh.n_hidden + 1;
    for (uint32_t l = 0; l < L; ++l) {
        const size_t ne = layer_elems(a.sh, l, a.kind);
        const uint32_t rows = layer_out(a.sh, l, a.kind);
        uint8_t *wdst = a.ws + a.lay.layer_w_off[l];
        float *bdst = reinterpret_cast<float *>(a.ws + a.lay.layer_b_off[l]);
        for (size_t e = tid; e < ne; e += stride) {
            float v;
            if (a.kind == MLP_VALU_F32) {
                const uint32_t cols = layer_in(a.sh, l);
                v = param_w(a, l, (int)(e / cols), (int)(e % cols));
            } else {
                const uint32_t P = mfma_p(a.kind);
                const uint32_t KC = layer_kchunks(a.sh, l, a.kind);
                const uint32_t p = e % P;
                const uint32_t lane = (e / P) % 64;
                const uint32_t kc = (e / (P * 64)) % KC;
                const uint32_t mb = e / ((size_t)P * 64 * KC);
                const int in = mfma_in_unit(a.sh, l, a.kind, kc, lane / 16, p);
                v = param_w(a, l, (int)(16 * mb + lane % 16), in);
            }
            if (a.kind == MLP_MFMA_F16) reinterpret_cast<_Float16 *>(wdst)[e] = (_Float16)v;
            else if (a.kind == MLP_MFMA_BF16) reinterpret_cast<uint16_t *>(wdst)[e] = float_to_bf16_rne(v);
            else reinterpret_cast<float *>(wdst)[e] = v;
        }
        for (uint32_t o = tid; o < rows; o += stride) bdst[o] = param_b(a, l, o);
    }
}

hipError_t launch_prepare_weights(const float *params, const MlpShape &sh, MlpKind kind,
                                  const WsLayout &lay, void *ws, hipStream_t s)
{
    PrepareArgs a{params, sh, kind, lay, static_cast<uint8_t *>(ws)};
    k_prepare<<<16, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// trilinear filtering from the texel scratch

struct LevelView {          // what one lane needs about its texture
    uint32_t w, h, levels;
    float bias;
    const uint32_t *tex_off;
};

__device__ __forceinline__ void bilinear(const uint2 *__restrict__ texels, const LevelView &T,
                                         uint32_t l, float uf, float vf, float out[3])
{
    const uint32_t w = max(T.w >> l, 1u), h = max(T.h >> l, 1u);
    const float x = fmaf(uf, (float)w, -0.5f), y = fmaf(vf, (float)h, -0.5f);
    const float xf = floorf(x), yf = floorf(y);
    const float fx = x - xf, fy = y - yf;
    const int ix = (int)xf, iy = (int)yf;
    const uint32_t x0 = (uint32_t)ix & (w - 1), x1 = (uint32_t)(ix + 1) & (w - 1);
    const uint32_t y0 = (uint32_t)iy & (h - 1), y1 = (uint32_t)(iy + 1) & (h - 1);
    const uint2 *base = texels + T.tex_off[l];
    const uint2 t00 = base[y0 * w + x0], t10 = base[y0 * w + x1];
    const uint2 t01 = base[y1 * w + x0], t11 = base[y1 * w + x1];
    const uint32_t a[4][2] = {{t00.x, t00.y}, {t10.x, t10.y}, {t01.x, t01.y}, {t11.x, t11.y}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t sh = c == 1 ? 16u : 0u;
        const int wd = c == 2 ? 1 : 0;
        const float v00 = half_bits_to_float((a[0][wd] >> sh) & 0xFFFFu);
        const float v10 = half_bits_to_float((a[1][wd] >> sh) & 0xFFFFu);
        const float v01 = half_bits_to_float((a[2][wd] >> sh) & 0xFFFFu);
        const float v11 = half_bits_to_float((a[3][wd] >> sh) & 0xFFFFu);
        const float r0 = fmaf(fx, v10 - v00, v00);
        const float r1 = fmaf(fx, v11 - v01, v01);
        out[c] = fmaf(fy, r1 - r0, r0);
    }
}

__device__ __forceinline__ void trilinear(const uint2 *__restrict__ texels, const LevelView &T,
                                          float u, float v, float s, float out[3])
{
    // scale s_i = s + b_i clamped to [0, L-1]; fmaxf maps NaN to 0
    const float si = fminf(fmaxf(s + T.bias, 0.0f), (float)(T.levels - 1));
    const float lf = floorf(si);
    const uint32_t l0 = (uint32_t)lf;
    const uint32_t l1 = min(l0 + 1, T.levels - 1);
    const float lam = si - lf;
    const float uf = u - floorf(u), vf = v - floorf(v);       // wrap addressing
    float a[3], b[3];
    bilinear(texels, T, l0, uf, vf, a);
    bilinear(texels, T, l1, uf, vf, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = fmaf(lam, b[c] - a[c], a[c]);
}

struct FilterMlpArgs {
    MaterialDesc m;
    const uint2 *texels;
    const uint8_t *ws;
    WsLayout lay;
    const float *queries;
    float *out;
    uint64_t n;
    uint32_t out_dim;
};

// ---------------------------------------------------------------------------
// plain fp32 path: one query per lane, every pyramid in turn, MLP on the
// vector ALU with wave-uniform (scalar) weight operands

template <int H, int NH, int C>
__global__ void __launch_bounds__(256) k_filter_mlp_valu(FilterMlpArgs a)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n; q += stride) {
        const float u = a.queries[3 * q], v = a.queries[3 * q + 1], s = a.queries[3 * q + 2];
        float z[12];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if ((uint32_t)t < a.m.n_tex) {
                const TexDesc &T = a.m.tex[t];
                LevelView lv{T.w, T.h, T.levels, T.bias, T.tex_off};
                trilinear(a.texels, lv, u, v, s, z + 3 * t);
            } else {
                z[3 * t] = z[3 * t + 1] = z[3 * t + 2] = 0.0f;
            }
        }
        // layer 0: H x 12
        const float *W = reinterpret_cast<const float *>(a.ws + a.lay.layer_w_off[0]);
        const float *B = reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[0]);
        float hcur[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float acc = B[j];
#pragma unroll
            for (int i = 0; i < 12; ++i) acc = fmaf(W[j * 12 + i], z[i], acc);
            hcur[j] = fmaxf(acc, 0.0f);
        }
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            W = reinterpret_cast<const float *>(a.ws + a.lay.layer_w_off[l]);
            B = reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[l]);
            float hn[H];
#pragma unroll
            for (int j = 0; j < H; ++j) {
                float acc = B[j];
#pragma unroll
                for (int i = 0; i < H; ++i) acc = fmaf(W[j * H + i], hcur[i], acc);
                hn[j] = fmaxf(acc, 0.0f);
            }
#pragma unroll
            for (int j = 0; j < H; ++j) hcur[j] = hn[j];
        }
        W = reinterpret_cast<const float *>(a.ws + a.lay.layer_w_off[NH]);
        B = reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[NH]);
        float *o = a.out + q * a.out_dim;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            float acc = B[j];
#pragma unroll
            for (int i = 0; i < H; ++i) acc = fmaf(W[j * H + i], hcur[i], acc);
            if ((uint32_t)j < a.out_dim) o[j] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA path: a wave decodes 16 queries; lane L filters pyramid L / 16 of
// query L % 16, which is the layer-0 B operand without any data movement.

template <MlpKind K> struct Mma;

template <> struct Mma<MLP_MFMA_F16> {
    static constexpr int P = 4;
    typedef half4_t Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return *reinterpret_cast<const half4_t *>(p + 2 * e);
    }
    static __device__ __forceinline__ Op pack(const float *x)
    {
        half4_t r = {(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
        return r;
    }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

template <> struct Mma<MLP_MFMA_BF16> {
    static constexpr int P = 4;
    typedef short4_t Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return *reinterpret_cast<const short4_t *>(p + 2 * e);
    }
    static __device__ __forceinline__ Op pack(const float *x)
    {
        short4_t r = {(short)float_to_bf16_rne(x[0]), (short)float_to_bf16_rne(x[1]),
                      (short)float_to_bf16_rne(x[2]), (short)float_to_bf16_rne(x[3])};
        return r;
    }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

template <> struct Mma<MLP_MFMA_F32> {
    static constexpr int P = 1;
    typedef float Op;
    static __device__ __forceinline__ Op load(const uint8_t *p, size_t e)
    {
        return reinterpret_cast<const float *>(p)[e];
    }
    static __device__ __forceinline__ Op pack(const float *x) { return x[0]; }
    static __device__ __forceinline__ float4_t mma(Op a, Op b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <MlpKind K, int H, int NH>
__global__ void __launch_bounds__(256) k_filter_mlp_mfma(FilterMlpArgs a)
{
    typedef Mma<K> M;
    constexpr int P = M::P;
    constexpr int HB = H / 16;                         // M blocks of a hidden layer
    constexpr int KC0 = P == 1 ? 3 : 1;                // K chunks of layer 0
    constexpr int KCH = P == 1 ? H / 4 : H / 16;       // K chunks of hidden inputs

    __shared__ uint32_t tex_lds[kMaxTextures][4 + kMaxLevels];
    for (int i = threadIdx.x; i < kMaxTextures * (4 + kMaxLevels); i += blockDim.x) {
        const int t = i / (4 + kMaxLevels), j = i % (4 + kMaxLevels);
        const TexDesc &T = a.m.tex[t];
        uint32_t v = 0;
        if (j == 0) v = T.w;
        else if (j == 1) v = T.h;
        else if (j == 2) v = T.levels;
        else if (j == 3) v = __builtin_bit_cast(uint32_t, T.bias);
        else v = T.tex_off[j - 4];
        tex_lds[t][j] = v;
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = lane >> 4, qi = lane & 15;
    const bool has_tex = g < a.m.n_tex;
    LevelView lv{tex_lds[g][0], tex_lds[g][1], tex_lds[g][2],
                 __builtin_bit_cast(float, tex_lds[g][3]), &tex_lds[g][4]};

    // weights and biases live in registers for the whole kernel
    typename M::Op w0[HB][KC0], wh[NH > 1 ? NH - 1 : 1][HB][KCH], wo[KCH];
    float4_t b0[HB], bh[NH > 1 ? NH - 1 : 1][HB], bo;
    {
        const uint8_t *p = a.ws + a.lay.layer_w_off[0];
        const float *bb = reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[0]);
#pragma unroll
        for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) w0[mb][kc] = M::load(p, ((size_t)(mb * KC0 + kc) * 64 + lane) * P);
            b0[mb] = *reinterpret_cast<const float4_t *>(bb + 16 * mb + 4 * g);
        }
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            const uint8_t *ph = a.ws + a.lay.layer_w_off[l];
            const float *bh_ = reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[l]);
#pragma unroll
            for (int mb = 0; mb < HB; ++mb) {
#pragma unroll
                for (int kc = 0; kc < KCH; ++kc)
                    wh[l - 1][mb][kc] = M::load(ph, ((size_t)(mb * KCH + kc) * 64 + lane) * P);
                bh[l - 1][mb] = *reinterpret_cast<const float4_t *>(bh_ + 16 * mb + 4 * g);
            }
        }
        const uint8_t *po = a.ws + a.lay.layer_w_off[NH];
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) wo[kc] = M::load(po, ((size_t)kc * 64 + lane) * P);
        bo = *reinterpret_cast<const float4_t *>(reinterpret_cast<const float *>(a.ws + a.lay.layer_b_off[NH]) + 4 * g);
    }

    const uint64_t n_groups = (a.n + 15) / 16;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t grp = wave; grp < n_groups; grp += n_waves) {
        const uint64_t q = grp * 16 + qi;
        float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (q < a.n && has_tex) {
            const float u = a.queries[3 * q], v = a.queries[3 * q + 1], s = a.queries[3 * q + 2];
            trilinear(a.texels, lv, u, v, s, f);
        }
        // layer 0
        typename M::Op x0[KC0];
        if (P == 1) {
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) x0[kc] = M::pack(f + kc);
        } else {
            x0[0] = M::pack(f);
        }
        float act[HB][4];
#pragma unroll
        for (int mb = 0; mb < HB; ++mb) {
            float4_t acc = b0[mb];
#pragma unroll
            for (int kc = 0; kc < KC0; ++kc) acc = M::mma(w0[mb][kc], x0[kc], acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) act[mb][j] = fmaxf(acc[j], 0.0f);
        }
        // hidden layers
#pragma unroll
        for (int l = 1; l < NH; ++l) {
            typename M::Op xin[KCH];
#pragma unroll
            for (int kc = 0; kc < KCH; ++kc) xin[kc] = P == 1 ? M::pack(&act[kc / 4][kc % 4]) : M::pack(act[kc]);
#pragma unroll
            for (int mb = 0; mb < HB; ++mb) {
                float4_t acc = bh[l - 1][mb];
#pragma unroll
                for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wh[l - 1][mb][kc], xin[kc], acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) act[mb][j] = fmaxf(acc[j], 0.0f);
            }
        }
        // output layer (one M block of 16 units)
        typename M::Op xin[KCH];
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) xin[kc] = P == 1 ? M::pack(&act[kc / 4][kc % 4]) : M::pack(act[kc]);
        float4_t acc = bo;
#pragma unroll
        for (int kc = 0; kc < KCH; ++kc) acc = M::mma(wo[kc], xin[kc], acc);
        if (q < a.n) {
            float *o = a.out + q * a.out_dim;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * g + j < a.out_dim) o[4 * g + j] = acc[j];
        }
    }
}

// ---------------------------------------------------------------------------
// dispatch

template <MlpKind K>
static hipError_t launch_mfma_kind(const FilterMlpArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s)
{
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        k_filter_mlp_mfma<K, H, NH><<<grid, 256, 0, s>>>(a);                                  \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

static hipError_t launch_valu(const FilterMlpArgs &a, const MlpShape &sh, hipStream_t s)
{
    const unsigned grid = (unsigned)std::min<uint64_t>((a.n + 255) / 256, 256u * 64u);
#define BCF_CASE(H, NH, C)                                                                    \
    if (sh.hidden == H && sh.n_hidden == NH && (C == 16 ? sh.out > 10 : sh.out <= 10)) {     \
        k_filter_mlp_valu<H, NH, C><<<grid, 256, 0, s>>>(a);                                  \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1, 10) BCF_CASE(16, 2, 10) BCF_CASE(16, 3, 10)
    BCF_CASE(32, 1, 10) BCF_CASE(32, 2, 10) BCF_CASE(32, 3, 10)
    BCF_CASE(64, 1, 10) BCF_CASE(64, 2, 10) BCF_CASE(64, 3, 10)
    BCF_CASE(16, 1, 16) BCF_CASE(16, 2, 16) BCF_CASE(16, 3, 16)
    BCF_CASE(32, 1, 16) BCF_CASE(32, 2, 16) BCF_CASE(32, 3, 16)
    BCF_CASE(64, 1, 16) BCF_CASE(64, 2, 16) BCF_CASE(64, 3, 16)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_filter_mlp(const MaterialDesc &m, const MlpShape &sh, MlpKind kind,
                             const WsLayout &lay, const void *ws, const float *queries, size_t n,
                             float *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    FilterMlpArgs a;
    a.m = m;
    a.ws = static_cast<const uint8_t *>(ws);
    a.texels = reinterpret_cast<const uint2 *>(a.ws + lay.scratch_off);
    a.lay = lay;
    a.queries = queries;
    a.out = out;
    a.n = n;
    a.out_dim = sh.out;
    if (kind == MLP_VALU_F32) return launch_valu(a, sh, s);
    const uint64_t groups = (n + 15) / 16;
    const unsigned grid = (unsigned)std::min<uint64_t>((groups + 3) / 4, 256u * 16u);
    switch (kind) {
    case MLP_MFMA_F16: return launch_mfma_kind<MLP_MFMA_F16>(a, sh, grid, s);
    case MLP_MFMA_BF16: return launch_mfma_kind<MLP_MFMA_BF16>(a, sh, grid, s);
    case MLP_MFMA_F32: return launch_mfma_kind<MLP_MFMA_F32>(a, sh, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bcf
