// Structures shared by the host API (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bcf {

constexpr int kMaxTextures = 4;
constexpr int kMaxLevels = 16;
constexpr int kMaxHidden = 64;
constexpr int kMaxOut = 16;
// queries per kernel launch: queries and outputs stay addressable with 32-bit
// byte offsets (at most 16 outputs of 4 bytes per query)
constexpr size_t kMaxQueriesPerLaunch = (size_t)1 << 25;

// One feature pyramid as the kernels see it.
struct TexDesc {
    const uint4 *blocks;            // level 0 block; levels follow back to back
    uint32_t w, h, levels;
    float bias;
    uint32_t blk_off[kMaxLevels];   // first block of each level
    uint32_t tex_off[kMaxLevels];   // first texel of each level in the texel scratch
};

struct MaterialDesc {
    TexDesc tex[kMaxTextures];
    uint32_t n_tex;
    uint32_t is_signed;
    // 1: the four pyramids share one geometry and their texel scratch is
    // position-packed -- texel (x, y) of level l of all four pyramids in one
    // 24-byte position of (r, g, b) halves (pyramid t at byte 6t), tex_off
    // counting positions and equal for every pyramid -- so a footprint row of
    // all four pyramids is one 48-byte span. 0: each pyramid's levels back to
    // back (8-byte texels (r | g << 16, b)).
    uint32_t interleaved;
};

// MLP arithmetic variants
enum MlpKind : uint32_t { MLP_VALU_F32 = 0, MLP_MFMA_F16 = 1, MLP_MFMA_BF16 = 2,
                          MLP_MFMA_FP8 = 3, MLP_MFMA_F32 = 4 };

// Shapes after padding: every hidden layer has `hidden` units (16, 32 or 64),
// the output has `out_pad` units (16 for MFMA, `out` rounded for VALU).
struct MlpShape {
    uint32_t n_hidden;              // hidden layers (1..3)
    uint32_t hidden;                // padded hidden width
    uint32_t out;                   // true output width (<= 16)
    uint32_t dims[5];               // true dims
    uint32_t n_layers;
};

// Workspace: weights of every layer in the kernel layout, then the texel scratch.
struct WsLayout {
    size_t weights_off, weights_bytes;
    size_t layer_w_off[4];          // byte offset of each layer's A-operand / matrix
    size_t layer_b_off[4];          // byte offset of each layer's fp32 bias (padded)
    size_t scales_off;              // fp32 per-layer dequantisation scales (fp8)
    size_t scratch_off, scratch_bytes;
    size_t total;
};

// The workspace bcf_decode_noalloc uses: a file-scope device array of
// kNoAllocBytes (noalloc.hip), one per GPU, held until the process ends.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
// its device address on the current device (looked up on the first call per device)
hipError_t noalloc_workspace(void **ptr);

// Kernel-side launchers (kernels.hip)
hipError_t launch_decode_blocks(const uint4 *blocks, size_t n, uint32_t is_signed, uint16_t *out,
                                hipStream_t s);

// Unpack segments: one per (pyramid, level), or one per level of an
// interleaved scratch (four lanes per block position, one per pyramid).
struct PredecodePlan {
    uint32_t n_seg;
    uint32_t seg_tex[kMaxTextures * kMaxLevels];
    uint32_t seg_lvl[kMaxTextures * kMaxLevels];
    uint32_t seg_wg[kMaxTextures * kMaxLevels + 1];     // first workgroup of each segment
};
hipError_t launch_predecode(const MaterialDesc &m, const PredecodePlan &p, uint2 *texels,
                            hipStream_t s);

// One segment of an unpack: one level of one pyramid, or of all four
// pyramids of a position-packed scratch (kSegInterleaved).
constexpr uint32_t kSegInterleaved = 1u, kSegSigned = 2u;
struct UnpackSeg {
    const uint4 *blocks[kMaxTextures];  // the level's first block per pyramid slot (slot 0 unless interleaved)
    uint2 *texels;                      // the level's first texel (interleaved: first position)
    uint32_t lw, lh;                    // level size in texels
    uint32_t wg0;                       // the segment's first chunk of 256 lanes in its launch
    uint32_t flags;                     // kSegInterleaved | kSegSigned
};
// every segment of a batch in one launch (segs in device memory, by first chunk)
// chunk_seg[c] = the segment of chunk c (n_chunks entries)
hipError_t launch_predecode_batch(const UnpackSeg *segs, const uint32_t *chunk_seg, uint32_t n_chunks, hipStream_t s);
// Unpacks the marked block positions of the interleaved segments and every
// chunk of the others: units[u] = first chunk of unit u (a window of up to
// four chunks of one interleaved segment, or one chunk of another segment).
hipError_t launch_predecode_touched(const UnpackSeg *segs, const uint32_t *chunk_seg, uint32_t n_seg,
                                    uint32_t n_chunks, const uint32_t *units, uint32_t n_units, const uint8_t *marks,
                                    hipStream_t s);
// Clears marks[0..mark_bytes) (a multiple of 16), fills the batch's item
// prefix, and marks the block positions the queries of the interleaved
// materials read.
hipError_t launch_batch_mark(void *ws, size_t table_off, size_t items_off, const float *queries,
                             const uint32_t *offsets, uint32_t n_mats, uint32_t n_total, uint8_t *marks,
                             size_t mark_bytes, hipStream_t s);

// operand elements and rows of layer l in the workspace (kernels.hip owns the layout)
size_t mlp_layer_elems(const MlpShape &s, uint32_t l, MlpKind k);
uint32_t mlp_layer_rows(const MlpShape &s, uint32_t l, MlpKind k);

// The first 256 bytes of a decode or batch workspace: what it was prepared
// for, so that a workspace describes itself (the host keeps the same tag per
// workspace address to validate later calls without reading device memory).
struct WsHeader {
    uint32_t magic;                 // kWsMagic
    uint32_t abi_version;
    uint32_t precision;             // bcf_precision
    uint32_t n_materials;           // 1 for a single-material workspace
    uint64_t layout_hash;           // the material(s) and precision it was prepared for
    uint64_t scratch_off, scratch_bytes;    // texel scratch (single material)
    uint64_t total_bytes;
};
constexpr uint32_t kWsMagic = 0x57464342u;   // "BCFW"

// header: written to the workspace's first bytes by the same launch (NULL: not written)
hipError_t launch_prepare_weights(const float *params, const float *act_absmax, const MlpShape &sh,
                                  MlpKind kind, const WsLayout &lay, void *ws, const WsHeader *header,
                                  hipStream_t s);

hipError_t launch_calibrate(const MaterialDesc &m, const MlpShape &sh, const WsLayout &lay, const void *ws,
                            const float *queries, size_t n, float *absmax, hipStream_t s);

// grid_width >= 8: the queries are an image of that many columns (row-major);
// results do not depend on it
hipError_t launch_filter_mlp(const MaterialDesc &m, const MlpShape &sh, MlpKind kind,
                             const WsLayout &lay, const void *ws, const float *queries, size_t n,
                             uint32_t grid_width, float *out, hipStream_t s);

// Many materials: where each material's texel scratch and MLP weights sit in
// the batch workspace.
struct BatchSlot {
    size_t scratch_off, scratch_bytes, weights_off;
    uint32_t seg_chunk[kMaxLevels];    // interleaved: first unpack chunk of each level's segment
};

size_t batch_table_bytes(uint32_t n_mats);
// builds the per-material table and copies it into the workspace (synchronises s)
// (and the header into the workspace's first bytes, table_off >= sizeof(WsHeader),
// the unpack segment table at segs_off, and the chunk map at chunk_seg_off)
hipError_t write_batch_table(const MaterialDesc *mats, const BatchSlot *slots, uint32_t n_mats, uint32_t out_dim,
                             const WsHeader &header, void *ws, size_t table_off, const UnpackSeg *segs,
                             uint32_t n_seg, size_t segs_off, const uint32_t *chunk_seg, uint32_t n_chunks,
                             size_t chunk_seg_off, hipStream_t s);
// Launch shape of the batched decode: workgroups, waves per workgroup (2 or
// 4), and how the waves share the items (runs of 64 queries): interleaved
// runs of `run` consecutive items, or one contiguous range per wave.
struct BatchShape {
    unsigned workgroups;
    uint32_t interleave, run, waves;
};

// rel: the weight layout relative to a material's weights_off
hipError_t launch_batch(void *ws, size_t table_off, size_t items_off, const WsLayout &rel, const MlpShape &sh,
                        MlpKind kind, const float *queries, const uint32_t *offsets, uint32_t n_mats,
                        uint32_t n_total, float *out, const BatchShape &shape, hipStream_t s);

}  // namespace bcf
