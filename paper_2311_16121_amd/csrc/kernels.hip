// Decode kernels for gfx950 (MI355X).
//
//  k_decode_blocks   BC6H blocks -> half bit patterns, one lane per block
//  k_predecode       every block of every pyramid -> texel scratch
//  k_prepare         MLP parameters -> padded per-precision operand layout
//  k_fp8_scales      per-layer fp8 weight and activation scales
//  (k_frame and k_calibrate live in frame_kernels.hpp, instantiated per MLP
//   precision in frame_<precision>.hip)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "bc6h_device.hpp"
#include "frame_kernels.hpp"
#include "internal.hpp"

namespace bcf {

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ void load_table(uint32_t *lds)
{
    for (int i = threadIdx.x; i < kTableWords; i += blockDim.x) lds[i] = kTable[i];
    __syncthreads();
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
// every block -> texel scratch (layout in filter_device.hpp)

struct PredecodeArgs {
    MaterialDesc m;
    PredecodePlan p;
    uint2 *texels;
};

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
// Global-memory views of the scratch and of the blocks. Pointers that the
// batch kernel reads from its segment table are generic to the compiler,
// which would access them with flat instructions (a flat store also counts
// against the LDS wait counter, so every LDS read after one waits for the
// store); these casts keep every access a global one.
typedef __attribute__((address_space(1))) u32x4_t global_u32x4;
typedef __attribute__((address_space(1))) const u32x4_t global_block;
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u32x2_t global_texel;

// Two texels to the scratch as one 16-byte non-temporal store: the unpack
// never reads them back, and the decode that follows it runs faster when the
// unpack's writes have not been left dirty in the caches (measured on the
// frame benchmark's unpack-then-decode step).
__device__ __forceinline__ void store_pair(uint2 *dst, uint2 t0, uint2 t1)
{
    __builtin_nontemporal_store((u32x4_t){t0.x, t0.y, t1.x, t1.y}, (global_u32x4 *)dst);
}

typedef uint32_t u32x3_t __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(1))) u32x3_t global_u32x3;

// Two pyramids' texels of one position of a packed scratch, (r, g, b) halves
// each, as one 12-byte store (dst 4-byte aligned). NT: non-temporal. A single
// material's unpack stores ordinarily: the decode that reads the scratch next
// runs faster when the unpack's lines went through the caches (frame4k, 134
// MB of scratch: 161 -> 138 us for the decode, 44 -> 50 us for the unpack).
// A batch's unpacks, gigabytes of scratch, store non-temporally (batch64: the
// decode 2.85 -> 2.79 ms, the whole unpack 4.06 -> 3.45 ms).
template <bool NT>
__device__ __forceinline__ void store_packed_pair(uint32_t *dst, uint2 t0, uint2 t1)
{
    const u32x3_t v = {t0.x, (t0.y & 0xFFFFu) | (t1.x << 16), (t1.x >> 16) | (t1.y << 16)};
    if (NT) __builtin_nontemporal_store(v, (global_u32x3 *)dst);
    else *(global_u32x3 *)dst = v;
}

// One chunk (256 lanes) of one unpack segment into the texel scratch. The
// whole workgroup calls it (it synchronises once); `palette` and `slots` are
// the workgroup's LDS, `table` the mode table. With `list` (LDS, interleaved
// segments only) the chunk is instead the block positions list[0..n_list)
// of the segment (at most 64), four lanes each; `chunk` is then unused.
template <bool SIGNED, bool NT>
__device__ __forceinline__ void unpack_chunk(const UnpackSeg &sg, uint32_t chunk, const uint32_t *table,
                                             uint2 (*palette)[256], uint2 *slots, const uint32_t *list = nullptr,
                                             uint32_t n_list = 0)
{
    // interleaved scratch: lane = 4 * block + pyramid, all four pyramids of a
    // level in one segment; otherwise lane = block of the segment's pyramid
    const uint32_t il = sg.flags & kSegInterleaved;
    const uint32_t li = list ? threadIdx.x : chunk * 256 + threadIdx.x;
    const uint32_t lw = sg.lw, lh = sg.lh;
    const uint32_t bx = (lw + 3) / 4, by = (lh + 3) / 4, n_blk = bx * by;
    // level sizes are powers of two: block bj sits at (bj & bxm, bj >> bxs)
    const uint32_t bxm = bx - 1u, bxs = (uint32_t)__builtin_ctz(bx);
    const uint32_t first = chunk * 256;         // this chunk's first block (per-pyramid layout)
    // a lane's block and whether it has one
    const bool have = list ? (threadIdx.x >> 2) < n_list : (il ? li >> 2 : li) < n_blk;
    const uint32_t bi = list ? (have ? list[threadIdx.x >> 2] : 0u) : (il ? li >> 2 : li);
    if (have) {
        // the lane's pyramid by selects (an indexed pointer array would sit
        // in private memory)
        const uint32_t pyr = il ? (li & 3u) : 0u;
        const uint4 *src = pyr == 0 ? sg.blocks[0] : pyr == 1 ? sg.blocks[1] : pyr == 2 ? sg.blocks[2] : sg.blocks[3];
        const u32x4_t b = ((global_block *)src)[bi];
        Bc6hHeader h;
        bc6h_header<SIGNED>(b.x, b.y, b.z, b.w, table, h);
        uint32_t pal[16][2];
        bc6h_palette<SIGNED>(h, pal);
#pragma unroll
        for (int j = 0; j < 16; ++j) palette[j][threadIdx.x] = make_uint2(pal[j][0], pal[j][1]);
        uint32_t s0, s1;
        bc6h_slots(h, s0, s1);
        slots[threadIdx.x] = make_uint2(s0, s1);
    }
    __syncthreads();
    const uint32_t pitch = row_pitch(lw);
    auto texel = [&](uint32_t lb, uint32_t t) {     // texel t (row-major) of the block in lane lb
        const uint2 sl = slots[lb];
        const uint32_t j = ((t < 8 ? sl.x : sl.y) >> (4 * (t & 7))) & 15u;
        return palette[j][lb];
    };
    if (il) {
        // A wave holds 16 blocks (four lanes each, one per pyramid). Each
        // block row is four 24-byte positions, 96 contiguous bytes; a store
        // instruction writes eight block rows: lane L takes the 12 bytes of
        // pyramids 2(L%2) and 2(L%2)+1 at position L % 8 / 2 of the row of
        // block 8h + L / 8, read through LDS from that block's lanes.
        // The store policy: store_packed_pair.
        uint32_t *pdst = reinterpret_cast<uint32_t *>(sg.texels);
        const uint32_t lane = threadIdx.x & 63u, wave0 = threadIdx.x & ~63u;
        const uint32_t chunk8 = lane & 7u, pp = 2 * (lane & 1u), cpos = chunk8 >> 1;
        for (uint32_t h = 0; h < 2; ++h) {
            const uint32_t blw = 8 * h + (lane >> 3);                     // block within the wave
            const uint32_t p = (wave0 >> 2) + blw;                        // within the chunk
            if (list ? p >= n_list : ((li - lane) >> 2) + blw >= n_blk) continue;
            const uint32_t bj = list ? list[p] : ((li - lane) >> 2) + blw;   // its index in the level
            const uint32_t lb = wave0 + 4 * blw + pp;                     // LDS lane of pyramid pp
            const uint32_t x0 = 4 * (bj & bxm), y0 = 4 * (bj >> bxs);
            for (uint32_t r = 0; r < 4; ++r) {
                if (y0 + r >= lh) break;
                // position index within the level (below 2^31: levels are at most 32768^2)
                const uint32_t prow = __umul24(y0 + r, pitch);
                // lw >= 4: texel column cpos; lw = 2: columns 0 1 0 1 (pitch 4);
                // lw = 1: texel 0 at positions 0 1 2 (pitch 3)
                if (lw == 1 && cpos >= 3) continue;
                const uint32_t col = lw >= 4 ? cpos : lw == 2 ? (cpos & 1u) : 0u;
                const uint2 p0 = texel(lb, 4 * r + col), p1 = texel(lb + 1, 4 * r + col);
                store_packed_pair<NT>(pdst + 6 * (size_t)(prow + x0 + cpos) + 3 * (pp >> 1), p0, p1);
                if (lw >= 4 && x0 == 0 && cpos < 2)                        // wrap positions w, w + 1
                    store_packed_pair<NT>(pdst + 6 * (size_t)(prow + lw + cpos) + 3 * (pp >> 1), p0, p1);
            }
        }
        return;
    }
    uint2 *dst = sg.texels;
    if (lw >= 4) {
        // A wave's 64 blocks, 32 at a time: lanes 2k and 2k + 1 write the
        // two halves of one block row, so each store instruction covers
        // whole 32-byte block rows (consecutive blocks of a block row are
        // contiguous). The level starts on a multiple of 4 texels and
        // pitch = w + 2 is even, so every store is 16-byte aligned.
        const uint32_t lane = threadIdx.x & 63, half = lane & 1;
#pragma unroll
        for (uint32_t g = 0; g < 2; ++g) {
            const uint32_t lb = (threadIdx.x & ~63u) + 32 * g + (lane >> 1);
            const uint32_t bj = first + lb;
            if (bj >= n_blk) continue;
            const uint32_t x0 = 4 * (bj & bxm), y0 = 4 * (bj >> bxs);
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                if (y0 + r >= lh) break;          // a level shorter than 4 texels
                const uint2 p0 = texel(lb, 4 * r + 2 * half), p1 = texel(lb, 4 * r + 2 * half + 1);
                const uint32_t trow = __umul24(y0 + r, pitch);   // texel index, below 2^31
                store_pair(dst + (trow + x0 + 2 * half), p0, p1);
                if (x0 == 0 && half == 0)         // wrap columns w and w+1: texels 0 and 1
                    store_pair(dst + (trow + lw), p0, p1);
            }
        }
    } else if (bi < n_blk) {
        // a level narrower than 4 texels keeps only the left part of its
        // blocks (and, shorter than 4, the top part)
        const uint32_t y0 = 4 * (bi >> bxs);
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            if (y0 + r >= lh) break;
            uint2 *row = dst + __umul24(y0 + r, pitch);
            const uint2 p0 = texel(threadIdx.x, 4 * r), p1 = texel(threadIdx.x, 4 * r + 1);
            if (lw == 2) {                        // pitch 4: texels 0 1 0 1
                store_pair(row, p0, p1);
                store_pair(row + 2, p0, p1);
            } else {                              // pitch 3: texel 0 three times
                global_texel *g = (global_texel *)row;
                const u32x2_t v = {p0.x, p0.y};
                g[0] = v;
                g[1] = v;
                g[2] = v;
            }
        }
    }
}

// The unpack segment of (pyramid or interleaved slot set, level) of a single
// material's plan entry `seg`.
__device__ __forceinline__ UnpackSeg material_seg(const PredecodeArgs &a, uint32_t seg)
{
    const uint32_t l = a.p.seg_lvl[seg];
    const uint32_t il = a.m.interleaved;
    UnpackSeg sg;
    for (uint32_t t = 0; t < (uint32_t)kMaxTextures; ++t) {
        const TexDesc &T = a.m.tex[il ? (t < a.m.n_tex ? t : 0u) : a.p.seg_tex[seg]];
        sg.blocks[t] = T.blocks + T.blk_off[l];
    }
    const TexDesc &T0 = a.m.tex[il ? 0u : a.p.seg_tex[seg]];
    sg.lw = max(T0.w >> l, 1u);
    sg.lh = max(T0.h >> l, 1u);
    // 8-byte units per position: 3 packed, 1 per pyramid
    sg.texels = a.texels + (il ? 3u : 1u) * (size_t)T0.tex_off[l];
    sg.wg0 = a.p.seg_wg[seg];
    sg.flags = il ? kSegInterleaved : 0u;
    return sg;
}

template <bool SIGNED>
__global__ void __launch_bounds__(256) k_predecode(PredecodeArgs a)
{
    __shared__ uint32_t table[kTableWords];
    // each lane's block palette, entry-major so that lane L's entries sit in
    // consecutive 8-byte slots across lanes, and its 16 four-bit slots
    __shared__ uint2 palette[16][256];
    __shared__ uint2 slots[256];
    load_table(table);
    // segment of this workgroup (uniform scan over at most 64 entries)
    const uint32_t wg = blockIdx.x;
    uint32_t seg = 0;
    while (seg + 1 < a.p.n_seg && a.p.seg_wg[seg + 1] <= wg) ++seg;
    const UnpackSeg sg = material_seg(a, seg);
    unpack_chunk<SIGNED, false>(sg, wg - sg.wg0, table, palette, slots);
}

// Every material of a batch in one launch: workgroup c unpacks chunk c of
// the segment table (and c + gridDim.x, ... when the table holds more chunks
// than one grid), its segment read from the chunk map (two dependent scalar
// loads; a search over the table costs a load per step, on every
// workgroup). One chunk per workgroup lets the hardware start a workgroup as
// soon as another retires, which keeps the stores of one chunk in flight
// beside the loads of the next (a persistent loop serialises them).
__global__ void __launch_bounds__(256) k_predecode_batch(const UnpackSeg *segs, const uint32_t *chunk_seg,
                                                         uint32_t n_chunks)
{
    __shared__ uint32_t table[kTableWords];
    __shared__ uint2 palette[16][256];
    __shared__ uint2 slots[256];
    load_table(table);
    for (uint32_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const UnpackSeg sg = segs[chunk_seg[c]];
        if (sg.flags & kSegSigned) unpack_chunk<true, true>(sg, c - sg.wg0, table, palette, slots);
        else unpack_chunk<false, true>(sg, c - sg.wg0, table, palette, slots);
        __syncthreads();                          // palette and slots are reused by the next chunk
    }
}

// The blocks of a batch that a set of queries touches, unpacked in one
// launch. Workgroup u takes unit units[u]: for a position-interleaved
// segment, a window of up to four chunks (256 block positions) whose marked
// positions it gathers in LDS and unpacks, 64 positions per pass (most
// windows need one pass with one or two busy waves); for any other segment,
// one whole chunk. marks[64 c + p] != 0: position p of chunk c is needed.
__global__ void __launch_bounds__(256) k_predecode_touched(const UnpackSeg *segs, const uint32_t *chunk_seg,
                                                           uint32_t n_seg, uint32_t n_chunks, const uint32_t *units,
                                                           uint32_t n_units, const uint8_t *marks)
{
    __shared__ uint32_t table[kTableWords];
    __shared__ uint2 palette[16][256];
    __shared__ uint2 slots[256];
    __shared__ uint32_t list[256];
    __shared__ uint32_t counts[4];
    load_table(table);
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    for (uint32_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const uint32_t c0 = units[u];
        const uint32_t sidx = chunk_seg[c0];
        const UnpackSeg sg = segs[sidx];
        const bool sgn = (sg.flags & kSegSigned) != 0;
        if (!(sg.flags & kSegInterleaved)) {
            if (sgn) unpack_chunk<true, true>(sg, c0 - sg.wg0, table, palette, slots);
            else unpack_chunk<false, true>(sg, c0 - sg.wg0, table, palette, slots);
            __syncthreads();                      // palette and slots are reused by the next unit
            continue;
        }
        const uint32_t end = sidx + 1 < n_seg ? segs[sidx + 1].wg0 : n_chunks;
        const uint32_t nc = min(4u, end - c0);
        const bool m = t < 64u * nc && marks[64ull * c0 + t] != 0;
        const uint64_t bal = __ballot(m);
        if (lane == 0) counts[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (uint32_t w = 0; w < 4; ++w) {
            const uint32_t c = counts[w];
            before += w < wv ? c : 0u;
            total += c;
        }
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (m) list[before + rank] = 64u * (c0 - sg.wg0) + t;       // the position within the segment
        __syncthreads();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t n = min(64u, total - p0);
            if (sgn) unpack_chunk<true, true>(sg, 0, table, palette, slots, list + p0, n);
            else unpack_chunk<false, true>(sg, 0, table, palette, slots, list + p0, n);
            __syncthreads();
        }
    }
}

hipError_t launch_predecode_touched(const UnpackSeg *segs, const uint32_t *chunk_seg, uint32_t n_seg,
                                    uint32_t n_chunks, const uint32_t *units, uint32_t n_units, const uint8_t *marks,
                                    hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    const unsigned grid = std::min<unsigned>(n_units, 1u << 22);
    k_predecode_touched<<<grid, 256, 0, s>>>(segs, chunk_seg, n_seg, n_chunks, units, n_units, marks);
    return hipGetLastError();
}

hipError_t launch_predecode_batch(const UnpackSeg *segs, const uint32_t *chunk_seg, uint32_t n_chunks, hipStream_t s)
{
    if (n_chunks == 0) return hipSuccess;
    // a grid of at most 2^22 workgroups (2^30 threads); larger tables loop
    const unsigned grid = std::min<unsigned>(n_chunks, 1u << 22);
    k_predecode_batch<<<grid, 256, 0, s>>>(segs, chunk_seg, n_chunks);
    return hipGetLastError();
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
// MLP operand layouts (see mlp_device.hpp for the MFMA slot order)
//
// VALU: layer l is W[rows][cols] fp32 row-major then b[rows], rows/cols padded
// (layer 0 cols = 12: z0 index 3 * pyramid + channel).
// MFMA: per layer [mblock][kchunk][lane][P] operand elements; the bias stays
// fp32 in natural order, padded to the M blocks.

__host__ __device__ inline uint32_t mfma_p(MlpKind k) { return k == MLP_MFMA_F32 ? 1u : 8u; }

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
    return l == 0 ? 1u : (s.hidden + 31) / 32;
}

// logical input unit of K slot (kc, g, p) of layer l, or -1 for padding
__host__ __device__ inline int mfma_in_unit(uint32_t l, MlpKind k, uint32_t kc, uint32_t g, uint32_t p)
{
    if (k == MLP_MFMA_F32) {
        if (l == 0) return (kc < 3) ? (int)(3 * g + kc) : -1;
        return (int)(16 * (kc / 4) + 4 * g + kc % 4);
    }
    if (l == 0) return p < 3 ? (int)(3 * g + p) : -1;
    return (int)(16 * (2 * kc + p / 4) + 4 * g + p % 4);
}

__host__ __device__ inline size_t layer_elems(const MlpShape &s, uint32_t l, MlpKind k)
{
    if (k == MLP_VALU_F32) return (size_t)layer_out(s, l, k) * layer_in(s, l);
    return (size_t)(layer_out(s, l, k) / 16) * layer_kchunks(s, l, k) * 64 * mfma_p(k);
}

size_t mlp_layer_elems(const MlpShape &s, uint32_t l, MlpKind k) { return layer_elems(s, l, k); }
uint32_t mlp_layer_rows(const MlpShape &s, uint32_t l, MlpKind k) { return layer_out(s, l, k); }

struct PrepareArgs {
    const float *params;
    const float *act_absmax;     // fp8: largest |input| of each layer (device)
    MlpShape sh;
    MlpKind kind;
    WsLayout lay;
    uint8_t *ws;
    WsHeader header;
    uint32_t write_header;
};

__device__ inline size_t param_offset(const MlpShape &sh, uint32_t l)
{
    size_t off = 0;
    for (uint32_t j = 0; j < l; ++j) off += (size_t)sh.dims[j] * sh.dims[j + 1] + sh.dims[j + 1];
    return off;
}

// true-layout parameter W_l[o][i] (0 outside the true shape)
__device__ inline float param_w(const PrepareArgs &a, uint32_t l, int o, int i)
{
    const uint32_t n_in = a.sh.dims[l], n_out = a.sh.dims[l + 1];
    if (o < 0 || i < 0 || (uint32_t)o >= n_out || (uint32_t)i >= n_in) return 0.0f;
    return a.params[param_offset(a.sh, l) + (size_t)o * n_in + i];
}

__device__ inline float param_b(const PrepareArgs &a, uint32_t l, uint32_t o)
{
    const uint32_t n_in = a.sh.dims[l], n_out = a.sh.dims[l + 1];
    return o < n_out ? a.params[param_offset(a.sh, l) + (size_t)n_in * n_out + o] : 0.0f;
}

// fp8 scales, one workgroup per layer. Scales region (floats): [2l] the
// accumulator's dequantisation factor s_w * s_a, [2l+1] 1 / s_a for the
// layer's input, [16 + l] 1 / s_w for the weight conversion, where
// s_w = max|W_l| / 448 and s_a = (largest |input|) / 448.
__global__ void __launch_bounds__(256) k_fp8_scales(PrepareArgs a)
{
    __shared__ float red[256];
    const uint32_t l = blockIdx.x;
    const uint32_t n = a.sh.dims[l] * a.sh.dims[l + 1];
    const float *W = a.params + param_offset(a.sh, l);
    float m = 0.0f;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fabsf(W[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (uint32_t s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float tiny = 1e-30f;
        const float sw = fmaxf(red[0], tiny) / kFp8Max;
        const float sa = fmaxf(a.act_absmax[l], tiny) / kFp8Max;
        float *sc = reinterpret_cast<float *>(a.ws + a.lay.scales_off);
        sc[2 * l] = sw * sa;
        sc[2 * l + 1] = 1.0f / sa;
        sc[16 + l] = 1.0f / sw;
    }
}

__global__ void k_prepare(PrepareArgs a)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t L = a.sh.n_hidden + 1;
    const float *sc = reinterpret_cast<const float *>(a.ws + a.lay.scales_off);
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
                const int in = mfma_in_unit(l, a.kind, kc, lane / 16, p);
                v = param_w(a, l, (int)(16 * mb + lane % 16), in);
            }
            if (a.kind == MLP_MFMA_F16) {
                reinterpret_cast<_Float16 *>(wdst)[e] = (_Float16)v;
            } else if (a.kind == MLP_MFMA_BF16) {
                reinterpret_cast<__bf16 *>(wdst)[e] = (__bf16)v;
            } else if (a.kind == MLP_MFMA_FP8) {
                wdst[e] = (uint8_t)(fp8x4(v * sc[16 + l], 0.0f, 0.0f, 0.0f) & 0xFFu);
            } else {
                reinterpret_cast<float *>(wdst)[e] = v;
            }
        }
        for (uint32_t o = tid; o < rows; o += stride) bdst[o] = param_b(a, l, o);
    }
    if (a.write_header && tid == 0) *reinterpret_cast<WsHeader *>(a.ws) = a.header;
}

hipError_t launch_prepare_weights(const float *params, const float *act_absmax, const MlpShape &sh,
                                  MlpKind kind, const WsLayout &lay, void *ws, const WsHeader *header,
                                  hipStream_t s)
{
    PrepareArgs a{params, act_absmax, sh, kind, lay, static_cast<uint8_t *>(ws), {}, 0u};
    if (header) {
        a.header = *header;
        a.write_header = 1;
    }
    if (kind == MLP_MFMA_FP8) {
        k_fp8_scales<<<sh.n_hidden + 1, 256, 0, s>>>(a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_prepare<<<16, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dispatch

__global__ void k_fill(float *p, uint32_t n, float v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Frame arguments common to the decode and the calibration.
// *layout: kLayoutPacked for a packed scratch, kLayoutShared for pyramids of
// one geometry a constant stride apart, else kLayoutSplit.
static FrameArgs frame_args(const MaterialDesc &m, const WsLayout &lay, const void *ws, uint32_t out_dim,
                            int *layout)
{
    FrameArgs a;
    std::memset(&a, 0, sizeof a);
    for (uint32_t t = 0; t < (uint32_t)kMaxTextures; ++t) {
        const TexDesc &T = m.tex[t < m.n_tex ? t : 0];   // unused slots repeat slot 0
        for (uint32_t l = 0; l < (uint32_t)kMaxLevels; ++l) {
            const uint32_t ll = l < T.levels ? l : T.levels - 1;
            const uint32_t w = std::max(T.w >> ll, 1u), h = std::max(T.h >> ll, 1u);
            const float fw = (float)w, fh = (float)h;
            uint4 e;
            std::memcpy(&e.x, &fw, 4);
            std::memcpy(&e.y, &fh, 4);
            e.z = (w - 1) | ((h - 1) << 16);
            e.w = T.tex_off[ll];
            a.lut.e[t][l] = e;
        }
        const uint32_t lv = T.levels;
        std::memcpy(&a.levels_bias[2 * t], &lv, 4);
        a.levels_bias[2 * t + 1] = T.bias;
    }
    // shared geometry: identical w, h, levels and bias, scratch a constant stride apart
    bool shared = true;
    const uint32_t stride_texels = m.n_tex > 1 ? m.tex[1].tex_off[0] - m.tex[0].tex_off[0] : 0;
    for (uint32_t t = 1; t < m.n_tex; ++t) {
        const TexDesc &A = m.tex[0], &B = m.tex[t];
        if (A.w != B.w || A.h != B.h || A.levels != B.levels || A.bias != B.bias) shared = false;
        for (uint32_t l = 0; l < A.levels && shared; ++l)
            if (B.tex_off[l] != A.tex_off[l] + t * stride_texels) shared = false;
    }
    *layout = m.interleaved ? kLayoutPacked : shared ? kLayoutShared : kLayoutSplit;
    a.stride = stride_texels * 8u;
    a.ws = static_cast<const uint8_t *>(ws);
    a.lay = lay;
    a.out_dim = out_dim;
    return a;
}

// The calibration's grid: at most 16 workgroups of 4 waves per CU, a multiple of the XCD count.
static unsigned frame_grid(uint32_t items)
{
    const uint32_t blocks = std::min<uint32_t>((items + kFrameWaves - 1) / kFrameWaves, 256u * 16u);
    return std::max(kXcds, (blocks + kXcds - 1) / kXcds * kXcds);
}

// tile rows per strip of a tiled frame (16 x 4 tiles: 16 image rows)
constexpr uint32_t kStripRows = 4;

hipError_t launch_filter_mlp(const MaterialDesc &m, const MlpShape &sh, MlpKind kind,
                             const WsLayout &lay, const void *ws, const float *queries, size_t n,
                             uint32_t grid_width, float *out, hipStream_t s)
{
    int layout;
    FrameArgs a = frame_args(m, lay, ws, sh.out, &layout);
    auto launch = [&]() -> hipError_t {
        switch (kind) {
        case MLP_VALU_F32: return launch_frame_f32(a, sh, layout, s);
        case MLP_MFMA_F16: return launch_frame_f16(a, sh, layout, s);
        case MLP_MFMA_BF16: return launch_frame_bf16(a, sh, layout, s);
        case MLP_MFMA_FP8: return launch_frame_fp8(a, sh, layout, s);
        case MLP_MFMA_F32: return launch_frame_f32_mfma(a, sh, layout, s);
        default: return hipErrorInvalidValue;
        }
    };
    if (grid_width >= kTileW && grid_width <= n && n <= kMaxQueriesPerLaunch) {
        // an image of grid_width columns: tiles of several rows, so a wave's
        // queries read overlapping texels in both directions
        const uint32_t rows = (uint32_t)((n + grid_width - 1) / grid_width);
        a.queries = queries;
        a.out = out;
        a.n = (uint32_t)n;
        a.grid_w = grid_width;
        a.tiles_x = (grid_width + kTileW - 1) / kTileW;
        a.tiles_y = (rows + kTileH - 1) / kTileH;
        a.n_items = a.tiles_x * a.tiles_y;
        // strips of kStripRows tile rows, fewer when the image has too few
        // tile rows to give every XCD a strip
        a.strip_rows = 0;
        for (uint32_t r = kStripRows; r >= 1 && !a.strip_rows; r /= 2)
            if (a.tiles_y >= r * kXcds) a.strip_rows = r;
        a.wide = (grid_width * sh.out) % 4 == 0 && (a.n * sh.out) % 4 == 0 && ((uintptr_t)out & 15) == 0;
        return launch();
    }
    // one launch covers at most kMaxQueriesPerLaunch queries (32-bit buffer offsets)
    for (size_t first = 0; first < n; first += kMaxQueriesPerLaunch) {
        const uint32_t cnt = (uint32_t)std::min<size_t>(n - first, kMaxQueriesPerLaunch);
        a.queries = queries + 3 * first;
        a.out = out + sh.out * first;
        a.n = cnt;
        a.n_items = (cnt + 63) / 64;
        a.tiles_x = kLinearRun;
        a.tiles_y = (a.n_items + kLinearRun - 1) / kLinearRun;
        a.strip_rows = a.tiles_y >= kXcds ? 1 : 0;
        a.wide = (cnt * sh.out) % 4 == 0 && ((uintptr_t)a.out & 15) == 0;
        const hipError_t e = launch();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// many materials

size_t batch_table_bytes(uint32_t n_mats) { return sizeof(BatchMat) * n_mats; }

// First work item of every material (runs of 64 queries): one wave, an
// exclusive prefix sum over 64 materials at a time.
__global__ void __launch_bounds__(64) k_batch_items(BatchArgs a)
{
    const uint32_t lane = threadIdx.x;
    uint32_t carry = 0;
    for (uint32_t k0 = 0; k0 < a.n_mats; k0 += 64) {
        const uint32_t k = k0 + lane;
        uint32_t cnt = 0;
        if (k < a.n_mats) {
            uint32_t q0, c;
            batch_range(a, k, q0, c);
            cnt = (c + 63u) / 64u;
        }
        uint32_t v = cnt;                         // inclusive scan across the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(v, d);
            if (lane >= (uint32_t)d) v += t;
        }
        if (k < a.n_mats) a.items[k] = carry + v - cnt;
        carry += __shfl(v, 63);
    }
    if (lane == 0) a.items[a.n_mats] = carry;
}

// Marks, for the position-packed materials of a batch, the block positions
// the queries' footprints read: the same work items, levels and taps as
// k_batch (items of 64 queries; a lane past a material's queries reads the
// query (0, 0, 0), as k_batch's does). marks[64 c + p] = 1 for position p of
// unpack chunk c. Byte stores: concurrent marks of one position store the
// same value. Each wave walks a contiguous range of items with its current
// material's level table in LDS, loading the next item's queries while it
// marks the current one's. The coarse levels (at most kPrivPositions block
// positions each, most of the footprints) are marked in a wave-private byte
// map in LDS and written out once per material the wave leaves.
constexpr uint32_t kPrivPositions = 4096, kPrivBytes = 8192;

__global__ void __launch_bounds__(256) k_batch_mark(BatchArgs a, uint8_t *marks)
{
    __shared__ uint4 lut[4][kMaxLevels];
    __shared__ uint32_t segc[4][kMaxLevels];
    __shared__ uint32_t poff[4][kMaxLevels], pcnt[4][kMaxLevels];   // private map: offset (~0: none), positions
    __shared__ uint32_t priv[4][kPrivBytes / 4];
    const uint32_t lane = threadIdx.x & 63u, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint8_t *pm = reinterpret_cast<uint8_t *>(priv[wv]);
    for (uint32_t i = lane; i < kPrivBytes / 4; i += 64) priv[wv][i] = 0u;
    const uint32_t total = a.items[a.n_mats];
    const uint32_t waves = gridDim.x * 4, w = blockIdx.x * 4 + wv;
    const uint32_t first = (uint32_t)((uint64_t)total * w / waves), end = (uint32_t)((uint64_t)total * (w + 1) / waves);
    if (first >= end) return;
    uint32_t lo = 0, hi = a.n_mats;                 // the material of `first`
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.items[mid] <= first) lo = mid;
        else hi = mid;
    }
    lo = uniform(lo);
    uint32_t base = 0, next = 0, interleaved = 0;
    float lb0 = 0.0f, lb1 = 0.0f;
    __amdgpu_buffer_rsrc_t rq = make_rsrc(a.queries, 0);
    auto enter = [&](uint32_t k) {                  // material k becomes current
        const BatchMat &M = a.mats[k];
        if (lane < (uint32_t)kMaxLevels) {
            lut[wv][lane] = M.lut.e[0][lane];
            segc[wv][lane] = M.seg_chunk[lane];
        }
        interleaved = uniform(M.interleaved);
        lb0 = __builtin_bit_cast(float, uniform(__builtin_bit_cast(uint32_t, M.levels_bias[0])));
        lb1 = __builtin_bit_cast(float, uniform(__builtin_bit_cast(uint32_t, M.levels_bias[1])));
        uint32_t q0, n_k;
        batch_range(a, k, q0, n_k);
        rq = make_rsrc(a.queries + 3ull * uniform(q0), uniform(n_k) * 12u);
        base = uniform(a.items[k]);
        next = uniform(a.items[k + 1]);
        wave_lds_sync();
        if (lane == 0) {                            // the private levels, coarsest first
            const uint32_t levels = __builtin_bit_cast(uint32_t, lb0);
            uint32_t used = 0;
            for (uint32_t l = kMaxLevels; l-- > 0;) {
                const uint32_t masks = lut[wv][l].z;
                const uint32_t n = (((masks & 0xFFFFu) + 4u) >> 2) * (((masks >> 16) + 4u) >> 2);
                const bool take = interleaved && l < levels && n <= kPrivPositions && used + n <= kPrivBytes;
                poff[wv][l] = take ? used : 0xFFFFFFFFu;
                pcnt[wv][l] = n;
                used += take ? n : 0u;
            }
        }
        wave_lds_sync();
    };
    auto flush = [&]() {                            // the private map to memory, cleared
        for (uint32_t l = 0; l < (uint32_t)kMaxLevels; ++l) {
            const uint32_t off = poff[wv][l];
            if (off == 0xFFFFFFFFu) continue;
            uint8_t *mk = marks + 64ull * segc[wv][l];
            for (uint32_t p = lane; p < pcnt[wv][l]; p += 64) {
                if (pm[off + p]) {
                    mk[p] = 1;
                    pm[off + p] = 0;
                }
            }
        }
        wave_lds_sync();
    };
    enter(lo);
    Query q = load_query(rq, (first - base) * 64 + lane);
    for (uint32_t it = first; it < end; ++it) {
        const uint32_t nx = it + 1;
        const bool same = nx < next;
        Query qn = Query{0.0f, 0.0f, 0.0f};
        if (nx < end && same) qn = load_query(rq, (nx - base) * 64 + lane);
        if (interleaved) {
            const float uf = q.u - floorf(q.u), vf = q.v - floorf(q.v);
            const LevelSel ls = select_levels(q.s, lb1, __builtin_bit_cast(uint32_t, lb0));
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t l = k ? ls.l1 : ls.l0;
                const TapCoords tc = tap_coords(lut[wv][l], uf, vf);
                const uint32_t bxn = (tc.wm + 4u) >> 2;                            // (w + 3) / 4
                const uint32_t xa = tc.x0 >> 2, xb = ((tc.x0 + 1u) & tc.wm) >> 2;   // column w is column 0
                const uint32_t ya = tc.y0 >> 2, yb = tc.y1 >> 2;
                // most footprints lie in one block: store each distinct position once
                const uint32_t off = poff[wv][l];
                auto mark = [&](uint8_t *mk) {
                    mk[ya * bxn + xa] = 1;
                    if (xb != xa) mk[ya * bxn + xb] = 1;
                    if (yb != ya) {
                        mk[yb * bxn + xa] = 1;
                        if (xb != xa) mk[yb * bxn + xb] = 1;
                    }
                };
                if (off != 0xFFFFFFFFu) mark(pm + off);           // LDS
                else mark(marks + 64ull * segc[wv][l]);          // memory
            }
        }
        if (nx < end && !same) {                    // the next item starts another material
            wave_lds_sync();                        // this item's LDS reads and marks are done
            flush();
            uint32_t k = lo + 1;
            while (k + 1 < a.n_mats && a.items[k + 1] <= nx) ++k;   // past empty materials
            lo = uniform(k);
            enter(lo);
            qn = load_query(rq, (nx - base) * 64 + lane);
        }
        q = qn;
    }
    wave_lds_sync();
    flush();
}

__global__ void __launch_bounds__(256) k_fill_u32x4(u32x4_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = (u32x4_t){0u, 0u, 0u, 0u};
}

hipError_t launch_batch_mark(void *ws, size_t table_off, size_t items_off, const float *queries,
                             const uint32_t *offsets, uint32_t n_mats, uint32_t n_total, uint8_t *marks,
                             size_t mark_bytes, hipStream_t s)
{
    // clear with a kernel (a graph replays it reliably), then the items, then the marks
    const size_t n16 = mark_bytes / 16;
    if (n16) {
        k_fill_u32x4<<<(unsigned)std::min<size_t>((n16 + 255) / 256, 8192), 256, 0, s>>>(
            reinterpret_cast<u32x4_t *>(marks), n16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.ws = static_cast<const uint8_t *>(ws);
    a.mats = reinterpret_cast<const BatchMat *>(static_cast<uint8_t *>(ws) + table_off);
    a.offsets = offsets;
    a.items = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(ws) + items_off);
    a.queries = queries;
    a.n_mats = n_mats;
    a.n_total = n_total;
    k_batch_items<<<1, 64, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // waves walk contiguous ranges of at least 16 items (1024 queries), at
    // most 8192 waves (what the chip keeps resident)
    const uint32_t items = (uint32_t)(((uint64_t)n_total + 63u) / 64u) + n_mats;
    const unsigned grid = std::min<unsigned>(std::max<unsigned>((items + 63u) / 64u, 1u), 2048u);
    k_batch_mark<<<grid, 256, 0, s>>>(a, marks);
    return hipGetLastError();
}

hipError_t write_batch_table(const MaterialDesc *mats, const BatchSlot *slots, uint32_t n_mats, uint32_t out_dim,
                             const WsHeader &header, void *ws, size_t table_off, const UnpackSeg *segs,
                             uint32_t n_seg, size_t segs_off, const uint32_t *chunk_seg, uint32_t n_chunks,
                             size_t chunk_seg_off, hipStream_t s)
{
    if (n_seg) {
        hipError_t e = hipMemcpyAsync(static_cast<uint8_t *>(ws) + segs_off, segs, sizeof(UnpackSeg) * n_seg,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(static_cast<uint8_t *>(ws) + chunk_seg_off, chunk_seg, sizeof(uint32_t) * n_chunks,
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
    }
    // the header at byte 0, then (from table_off) the material table: one copy
    std::vector<uint8_t> host(table_off + sizeof(BatchMat) * n_mats, 0);
    std::memcpy(host.data(), &header, sizeof header);
    BatchMat *table = reinterpret_cast<BatchMat *>(host.data() + table_off);
    for (uint32_t k = 0; k < n_mats; ++k) {
        WsLayout lay;
        std::memset(&lay, 0, sizeof lay);
        lay.scratch_off = slots[k].scratch_off;
        int layout;
        const FrameArgs a = frame_args(mats[k], lay, ws, out_dim, &layout);
        BatchMat &b = table[k];
        std::memset(&b, 0, sizeof b);
        b.lut = a.lut;
        std::memcpy(b.levels_bias, a.levels_bias, sizeof b.levels_bias);
        b.scratch_off = slots[k].scratch_off;
        b.weights_off = slots[k].weights_off;
        b.scratch_bytes = (uint32_t)slots[k].scratch_bytes;
        b.stride = a.stride;
        b.shared = layout != kLayoutSplit ? 1u : 0u;
        b.interleaved = mats[k].interleaved;
        std::memcpy(b.seg_chunk, slots[k].seg_chunk, sizeof b.seg_chunk);
    }
    hipError_t e = hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);           // the host tables go out of scope
}

hipError_t launch_batch(void *ws, size_t table_off, size_t items_off, const WsLayout &rel, const MlpShape &sh,
                        MlpKind kind, const float *queries, const uint32_t *offsets, uint32_t n_mats,
                        uint32_t n_total, float *out, const BatchShape &shape, hipStream_t s)
{
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.ws = static_cast<const uint8_t *>(ws);
    a.mats = reinterpret_cast<const BatchMat *>(static_cast<uint8_t *>(ws) + table_off);
    a.offsets = offsets;
    a.items = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(ws) + items_off);
    a.lay = rel;
    a.queries = queries;
    a.out = out;
    a.n_mats = n_mats;
    a.n_total = n_total;
    a.out_dim = sh.out;
    a.interleave = shape.interleave;
    a.run = shape.run;
    k_batch_items<<<1, 64, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t waves = shape.waves == 2 ? 2u : 4u;
    const unsigned cap = 256u * 64u / waves;               // at most 64 waves per CU's worth
    const unsigned grid = std::max(kXcds, (std::min(shape.workgroups, cap) + kXcds - 1) / kXcds * kXcds);
    switch (kind) {
    case MLP_MFMA_F16: return launch_batch_f16(a, sh, grid, waves, s);
    case MLP_VALU_F32: return launch_batch_f32(a, sh, grid, waves, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_calibrate(const MaterialDesc &m, const MlpShape &sh, const WsLayout &lay, const void *ws,
                            const float *queries, size_t n, float *absmax, hipStream_t s)
{
    k_fill<<<1, 64, 0, s>>>(absmax, sh.n_hidden + 1, 0.0f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int layout;
    FrameArgs a = frame_args(m, lay, ws, sh.out, &layout);
    a.absmax = absmax;
    for (size_t first = 0; first < n; first += kMaxQueriesPerLaunch) {
        const uint32_t cnt = (uint32_t)std::min<size_t>(n - first, kMaxQueriesPerLaunch);
        a.queries = queries + 3 * first;
        a.n = cnt;
        const unsigned grid = std::max(1u, std::min<uint32_t>((cnt + kFrameThreads - 1) / kFrameThreads, 1024u));
        e = launch_calibrate_kernel(a, sh, layout, grid, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bcf
