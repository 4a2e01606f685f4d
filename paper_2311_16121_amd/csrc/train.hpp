// Training-time decode (Section 4.2, "Trainable BC6 decompression"): the
// descriptors shared by the host API (train_api.cpp) and the kernels
// (train.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "internal.hpp"

namespace bcf {

constexpr int kTrainMaxHidden = 32;
// The backward takes its samples in spatial order: per call of at most
// kTrainBinBatch samples, a counting sort by cell of a kTrainBinSide^2 grid
// over the wrapped (u, v), the cells numbered along a Z-order curve.
constexpr uint32_t kTrainBinBatch = 1u << 20;
constexpr uint32_t kTrainBinSide = 64;
constexpr uint32_t kTrainBins = kTrainBinSide * kTrainBinSide;

// One pyramid of continuous two-subset blocks (6-bit endpoints, 3-bit
// indices, fixed partitions), all levels back to back.
struct TrainTexDesc {
    const float *endpoints;        // [n_blocks][4][3]
    const float *indices;          // [n_blocks][16]
    const uint8_t *partitions;     // [n_blocks]
    float *g_endpoints;            // backward outputs, same layouts
    float *g_indices;
    uint32_t w, h, levels;
    float bias;
    uint32_t n_blocks;
    uint32_t blk_off[kMaxLevels];  // first block of each level
    uint32_t tex_off[kMaxLevels];  // first texel of each level in the texel images (pitch w_l)
};

struct TrainDesc {
    TrainTexDesc tex[kMaxTextures];
    uint32_t n_tex;
    uint32_t ste;                  // 1: straight-through (exact decode forward)
    uint32_t blk_base[kMaxTextures + 1];   // first block of each pyramid in a joint numbering
    float4 *texels;                // texel values (r, g, b, 0)
    float4 *g_texels;              // their gradients
    uint32_t n_texels;
    const float *params;           // per layer W[out][in] row-major, then b[out]
    float *g_params;
    uint32_t n_params;
    uint32_t dims[5];
    uint32_t n_layers;
    uint32_t w_off[4], b_off[4];   // float offsets of each layer's W and b in params
    // the forward's MLP operands (workspace): the matrix-core layout of the
    // fp32 16x16x4 MFMAs, offsets from ops_ws
    MlpShape ops_shape;
    WsLayout ops;
    uint8_t *ops_ws;
    // the backward's sample sort (workspace): sorted sample indices, per-cell
    // counts, per-cell next free slot (after the sort: the end of the cell's
    // run), and dL/dz (12 floats) per sorted sample
    uint32_t *bin_perm, *bin_count, *bin_next;
    float *bin_dz;
};

hipError_t launch_train_forward(const TrainDesc &d, const float *queries, size_t n, float *out,
                                hipStream_t s);
hipError_t launch_train_backward(const TrainDesc &d, const float *queries, size_t n, const float *grad_out,
                                 hipStream_t s);

}  // namespace bcf
