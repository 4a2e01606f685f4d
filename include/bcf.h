/*
 * bcf.h -- C ABI of the block-compressed neural material decoder for AMD
 * Instinct MI355X (gfx950).
 *
 * Computes the neural material of Weinreich et al., "Real-Time Neural
 * Materials using Block-Compressed Features" (arXiv 2311.16121):
 *
 *     G(u, v, s) = f_eta(T_0(u, v, s_0), ..., T_{n-1}(u, v, s_{n-1}))      eq. (3)
 *
 * where every feature pyramid T_i is a mip chain of BC6H blocks (Section 4,
 * "Block Based Neural Features"; Section 5.2, "Real-time Decoding": the
 * exported features are mip-mapped BC6 textures and the MLP weights a small
 * binary buffer), T_i is filtered trilinearly (eq. 9) at s_i = s + b_i
 * (eq. 10), and f_eta is a ReLU MLP (Section 5.1, "Model structure").
 *
 * Conventions for every call:
 *  - "device" pointers are HIP device memory (e.g. from torch); "host"
 *    pointers are ordinary process memory read during the call only.
 *  - The caller owns every buffer. No call allocates device memory.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) and never synchronise the host. Kernel faults surface at the
 *    caller's next synchronisation.
 *  - A non-OK status leaves a thread-local description in bcf_last_error().
 *  - All entry points are thread-safe.
 */
#ifndef BCF_H
#define BCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BCF_ABI_VERSION 2

typedef enum {
    BCF_OK = 0,
    BCF_ERR_INVALID_ARG = 1,   /* argument validation failed */
    BCF_ERR_UNSUPPORTED = 2,   /* valid but outside what the kernels implement */
    BCF_ERR_DEVICE = 3         /* a HIP runtime call or kernel launch failed */
} bcf_status;

/* Arithmetic of the decoder MLP f_eta. Fetch, BC6H unpacking (exact integer
 * work) and trilinear filtering (binary32) are identical in every mode. */
typedef enum {
    BCF_FP32 = 0,       /* plain binary32 vector ALU MLP */
    BCF_FP16 = 1,       /* MFMA, fp16 weights and activations, fp32 accumulation */
    BCF_BF16 = 2,       /* MFMA, bf16 weights and activations, fp32 accumulation */
    BCF_FP8 = 3,        /* MFMA, OCP e4m3 weights and activations with per-layer
                           scales, fp32 accumulation; needs act_absmax */
    BCF_FP32_MFMA = 4   /* MFMA on binary32 operands, fp32 accumulation */
} bcf_precision;

/* One feature pyramid T_i (Section 4.3, "Hardware compliant filtering").
 * `blocks` (device, 16-byte aligned) holds levels 0..levels-1 back to back.
 * Level l covers max(width>>l,1) x max(height>>l,1) texels stored as a
 * row-major grid of 16-byte BC6H blocks (4x4 texels each, texel t of a block
 * at x = t&3, y = t>>2); a level smaller than 4x4 is one block whose
 * top-left texels are used. width and height are powers of two;
 * 1 <= levels <= log2(max(width, height)) + 1. Addressing wraps in u and v.
 * `lod_bias` is b_i of eq. (10). */
typedef struct {
    const void *blocks;
    uint32_t width, height;
    uint32_t levels;
    float lod_bias;
} bcf_texture;

/* A material: n_textures (1..4) three-channel pyramids whose filtered values
 * are concatenated in order into the MLP input z0 (eq. 3), and the decoder
 * f_eta with n_layers (2..4) linear layers of sizes dims[0..n_layers]:
 * dims[0] == 3 * n_textures, hidden sizes <= 64, output dims[n_layers] <= 16.
 * ReLU follows every layer but the last. `params` (device, binary32) holds
 * per layer W[dims[l+1]][dims[l]] row-major, then b[dims[l+1]].
 * is_signed selects BC6H_SF16 (1) or BC6H_UF16 (0) for every texture.
 * act_absmax (device, n_layers floats, or NULL) is the largest magnitude of
 * each layer's input over a calibration batch (bcf_calibrate); only BCF_FP8
 * reads it, to fix its static per-layer activation scales. */
typedef struct {
    uint32_t n_textures;
    const bcf_texture *textures;   /* host array [n_textures] */
    uint32_t n_layers;
    const uint32_t *dims;          /* host array [n_layers + 1] */
    const float *params;           /* device */
    uint32_t is_signed;
    const float *act_absmax;       /* device, may be NULL */
} bcf_material;

/* ABI version of the loaded library (BCF_ABI_VERSION). */
int bcf_abi_version(void);

/* Thread-local description of the last non-OK status on this thread. */
const char *bcf_last_error(void);

/* Bytes of a full `levels`-level chain of a width x height BC6H texture,
 * 16 bytes per 4x4 block (the storage rule behind Table 2's sizes).
 * Returns 0 for invalid sizes. */
size_t bcf_texture_bytes(uint32_t width, uint32_t height, uint32_t levels);

/* Workspace for decoding `m` at precision `p`: the decoder's weights in the
 * form the kernels read (Section 5.2 ships the MLP weights as a small fp16
 * binary beside the mip-mapped BC6 textures; this call builds that buffer,
 * at the chosen precision, from the binary32 parameters).
 * Size query: with ws == NULL, writes the required size (bytes, 256-byte
 * aligned start required) to *ws_bytes and returns.
 * Fill: with ws != NULL (device) and *ws_bytes >= the size, converts the MLP
 * parameters into the kernels' padded layout for `p` (rounding to fp16/bf16
 * or e4m3 with per-layer scales; binary32 stays exact) asynchronously on
 * `stream`, and writes a 256-byte header at ws (magic "BCFW", ABI version,
 * precision, a hash of the material's pyramid geometry, block and parameter
 * addresses and MLP shape, and the layout's offsets). The library also
 * remembers that tag per workspace address on the host: bcf_decode,
 * bcf_unpack, bcf_decode_unpacked and bcf_calibrate return
 * BCF_ERR_INVALID_ARG for a workspace that no bcf_prepare filled, or that
 * was prepared for another precision or another material, without reading
 * device memory. The workspace also holds the texel scratch that bcf_unpack
 * (and bcf_decode) WRITE and the decode reads, so one workspace serves one
 * decode at a time: two decodes that share a workspace must be ordered on
 * one stream. The material's parameter values must not change between
 * prepare and decode without preparing again, nor its textures without
 * unpacking again. */
bcf_status bcf_prepare(const bcf_material *m, bcf_precision p, void *ws,
                       size_t *ws_bytes, void *stream);

/* Decode n queries: queries (device, [n][3] binary32 (u, v, s)) ->
 * out (device, [n][dims[n_layers]] binary32, row-major). s is the scale of
 * eq. (9) before the per-texture bias. grid_width > 0 declares that the
 * queries are a row-major image of that many columns (a frame in scanline
 * order; the last row may be partial), which lets the decoder walk it in
 * small 2D tiles whose queries share texels; 0 means no 2D structure.
 * Results do not depend on grid_width.
 * n == 0 is a no-op. out must not overlap queries, ws or the material.
 * Non-finite query components produce unspecified values but never an
 * out-of-bounds access. Same as bcf_unpack followed by bcf_decode_unpacked
 * on `stream`: ws (prepared for `p` and this material) is written -- it
 * receives the unpacked texels -- so concurrent decodes need one workspace
 * each. */
bcf_status bcf_decode(const bcf_material *m, bcf_precision p, void *ws,
                      const float *queries, size_t n, uint32_t grid_width,
                      float *out, void *stream);

/* bcf_decode for callers that cannot allocate device memory -- code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation --
 * and so cannot provide the workspace bcf_prepare fills. The library holds
 * the workspace itself: one 64 MiB array per GPU (BCF_NOALLOC_BYTES), in
 * device memory the library's code object reserves when it is loaded and
 * keeps until the process ends. Each call prepares the MLP weights for `p`
 * into it, unpacks the material's blocks into it and decodes, on `stream`
 * (which must belong to the current device); queries, n, grid_width and out
 * as in bcf_decode. No call allocates or frees memory (the first call on a
 * device looks up the array's device address once).
 * Returns BCF_ERR_UNSUPPORTED, before any launch, for a material whose
 * workspace (texel scratch and MLP operands, the size bcf_prepare reports)
 * exceeds BCF_NOALLOC_BYTES -- up to four 1024 x 1024 pyramids with full
 * chains fit. All calls on one GPU share its array and leave their data in
 * it: calls that overlap in time on one GPU (other streams, other threads)
 * race and give undefined results; order them on one stream. */
#define BCF_NOALLOC_BYTES ((size_t)64 << 20)
bcf_status bcf_decode_noalloc(const bcf_material *m, bcf_precision p, const float *queries, size_t n,
                              uint32_t grid_width, float *out, void *stream);

/* First half of bcf_decode: unpacks every BC6H block of every level of every
 * pyramid (Section 4.2, eqs. (6)-(8) in the format's integer form) into the
 * texel scratch of ws (device, prepared for this material at any precision;
 * the scratch layout does not depend on the precision). The texels stay valid
 * until the textures change, so a material drawn several times between
 * texture updates needs one unpack. */
bcf_status bcf_unpack(const bcf_material *m, void *ws, void *stream);

/* Second half of bcf_decode: trilinear filtering (eqs. (9), (10)) of the
 * texels a previous bcf_unpack of this material left in ws, and the MLP
 * (eq. (3)), with bcf_decode's arguments and results. ws must have been
 * prepared for `p` and unpacked, in stream order, before this call. */
bcf_status bcf_decode_unpacked(const bcf_material *m, bcf_precision p, const void *ws,
                               const float *queries, size_t n, uint32_t grid_width,
                               float *out, void *stream);

/* Calibration for BCF_FP8 (Section 5.2 stores the MLP weights in a reduced
 * precision; fp8 also quantises activations, with static per-layer scales):
 * decodes n queries (device, [n][3]) with the plain fp32 path and writes to
 * act_absmax (device, n_layers floats) the largest magnitude each layer's
 * input reaches. `ws` must be a workspace prepared for BCF_FP32 for this
 * material (its texel scratch is overwritten). */
bcf_status bcf_calibrate(const bcf_material *m, void *ws, const float *queries, size_t n,
                         float *act_absmax, void *stream);

/* Unpack n BC6H blocks (device, [n][16] bytes, 16-byte aligned) to half-float
 * bit patterns (device, [n][16][3] uint16, texel-major, r g b), bit-exact per
 * the BC6H format definition (Section 4.2's eqs. (6)-(8) in the format's
 * integer form). Reserved mode codes decode to zeros. */
bcf_status bcf_decode_blocks(const void *blocks, size_t n_blocks, uint32_t is_signed,
                             uint16_t *halves, void *stream);

/* ------------------------------------------------------------------------
 * Many materials in one launch (Section 5.2 decodes every material of a frame
 * with its own features and weights; here all of them go through one
 * persistent kernel).
 *
 * A batch is an array of n_mats materials (1..4096) that share one MLP shape
 * (dims) and run at BCF_FP16 or BCF_FP32; pyramid sizes, level counts, biases
 * and signedness may differ. Material k's queries are rows offsets[k] ..
 * offsets[k+1]-1 of one concatenated query array, and its outputs the same
 * rows of out. offsets is a DEVICE array of n_mats + 1 uint32 values, read by
 * the kernels: a captured graph replays with whatever the caller has written
 * there since. The kernels clamp every offset to [0, n_total] (n_total = rows
 * of queries and out), treat a decreasing pair as an empty material and decode
 * at most 2^25 queries per material (the first 2^25 of a longer range); rows
 * no material covers are not written. Offsets are expected non-decreasing:
 * with a later offset below an earlier one, two materials' ranges can
 * overlap, and each then writes the shared rows, in unspecified order. The
 * calls that take a batch workspace return BCF_ERR_INVALID_ARG when it was
 * not filled by bcf_prepare_batch for these materials (and, for the decode
 * and the tuner, this precision).
 * ------------------------------------------------------------------------ */

/* Launch shape of bcf_decode_batch (bcf_tune_batch picks one). A work item
 * is a run of 64 consecutive queries of one material. */
typedef struct {
    uint32_t workgroups;   /* persistent workgroups (rounded up to a multiple of 8);
                              0 = a default from n_total */
    uint32_t interleave;   /* 1: the waves take interleaved runs of `run` items;
                              0: each wave one contiguous range of items */
    uint32_t run;          /* interleaved: consecutive items per wave turn (items of
                              64 x run queries); 0 means 1 */
    uint32_t waves;        /* waves per workgroup: 2 or 4 (0 means 4) */
} bcf_batch_plan;

/* Workspace bytes for the batch (256-byte aligned start). */
bcf_status bcf_batch_workspace_size(const bcf_material *mats, uint32_t n_mats, bcf_precision p,
                                    size_t *ws_bytes);

/* Converts every material's MLP into the workspace and writes the batch's
 * material table. Synchronises `stream` (the table is copied from host
 * memory); not for graph capture. */
bcf_status bcf_prepare_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws,
                             size_t ws_bytes, void *stream);

/* bcf_unpack for every material of the batch, in one launch (each workgroup
 * unpacks one 256-lane chunk of a table of every material's (pyramid, level)
 * segments that bcf_prepare_batch wrote into the workspace).
 * A material whose four pyramids share size, level count and bias keeps its
 * texels position-interleaved in the batch workspace (the four pyramids'
 * texels of one position together), so a decode reads one footprint row of
 * all four from one span; results do not depend on the layout. */
bcf_status bcf_unpack_batch(const bcf_material *mats, uint32_t n_mats, void *ws, void *stream);

/* bcf_unpack_batch restricted to the blocks that these queries' trilinear
 * footprints read (eqs. 9 and 10 at the queries' LODs), the way Section 5.2's
 * renderer decodes only the blocks its samples touch: a bcf_decode_batch
 * with the same queries and offsets, and no call in between that writes the
 * workspace, then returns exactly what it returns after bcf_unpack_batch.
 * Texels of other blocks keep whatever the workspace held, so a decode of
 * other queries needs its own unpack. queries, offsets and n_total as for
 * bcf_decode_batch (device memory; offsets read on the device). For the
 * position-interleaved materials the footprints' block positions are first
 * marked in a byte table of the workspace (three launches: clear, item
 * prefix, mark), then one launch unpacks the marked positions and every
 * block of the other materials. Asynchronous, no allocation or host
 * synchronisation: it can be captured in a graph with bcf_decode_batch.
 * Errors as for bcf_unpack_batch, and BCF_ERR_INVALID_ARG for NULL or
 * misaligned queries (n_total > 0) or offsets. */
bcf_status bcf_unpack_batch_touched(const bcf_material *mats, uint32_t n_mats, void *ws, const float *queries,
                                    const uint32_t *offsets, uint32_t n_total, void *stream);

/* Decodes every material's queries in one persistent launch (after a small
 * launch that turns offsets into work items). Asynchronous and free of host
 * synchronisation and allocation, so it can be captured in a graph together
 * with bcf_unpack_batch. plan may be NULL. */
bcf_status bcf_decode_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws,
                            const float *queries, const uint32_t *offsets, uint32_t n_total,
                            float *out, const bcf_batch_plan *plan, void *stream);

/* Autotuner: runs bcf_decode_batch over a set of launch shapes on these
 * inputs -- workgroup counts, 2 or 4 waves per workgroup, contiguous ranges
 * or interleaved runs of 1, 2 or 4 items (64, 128 or 256 queries) -- timing
 * each with events, and returns the fastest in *best (and its time in
 * *best_ms when not NULL). Synchronises `stream`; out is overwritten. */
bcf_status bcf_tune_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws,
                          const float *queries, const uint32_t *offsets, uint32_t n_total,
                          float *out, bcf_batch_plan *best, float *best_ms, void *stream);

/* ------------------------------------------------------------------------
 * Training-time decode (Section 4.2, "Trainable BC6 decompression"; the
 * training of eqs. (4)-(5) differentiates through it).
 *
 * A trainable pyramid keeps, per 4x4 block of every level, the continuous
 * parameters of the two-subset BC6H mode the features are exported in
 * (Section 5.2: 6-bit endpoints, 3-bit indices) and a fixed partition
 * (Section 5.1, "Partition selection strategy"):
 *   endpoints  e_1..e_4 per channel, in quantised units (valid range [0, 63])
 *   indices    x per texel (valid range [0, 1])
 *   partition  k in 0..31 (only the low 5 bits are read)
 * Texel t of a block lies in subset sigma = bit t of partition mask k and
 * blends the pair (e_{2 sigma + 1}, e_{2 sigma + 2}):
 *   continuous:        y = a ((2^16 e_A + 2^15) + x 2^16 (e_B - e_A)) / 2^6,
 *                      a = 31/64 (eqs. (6), (7)), texel = eq. (8) of y;
 *   straight-through:  texel = the format's exact decode of the block with
 *                      endpoints rounded to integers in [0, 63] and indices
 *                      to i = rint(7 x) in [0, 7] -- the exported block;
 *                      gradients as in the continuous case at the rounded
 *                      point (x = w_i / 64, w_i the format's 3-bit weight),
 *                      the rounding passed through as the identity, and
 *                      eq. (8)'s slope taken at the decoded half.
 * Filtering and the MLP are those of bcf_decode (eqs. (9), (10), (3)) in
 * binary32, with every hidden layer of 16 or 32 units.
 * ------------------------------------------------------------------------ */

typedef struct {
    uint32_t width, height;        /* powers of two */
    uint32_t levels;               /* 1 .. log2(max(width, height)) + 1 */
    float lod_bias;                /* b_i of eq. (10) */
    const float *endpoints;        /* device [n_blocks][4][3], levels back to back */
    const float *indices;          /* device [n_blocks][16] */
    const uint8_t *partitions;     /* device [n_blocks] */
} bcf_train_texture;

typedef struct {
    uint32_t n_textures;                  /* 1..4 */
    const bcf_train_texture *textures;    /* host array [n_textures] */
    uint32_t n_layers;                    /* 2..4 */
    const uint32_t *dims;                 /* host [n_layers + 1]; hidden widths 16 or 32 */
    const float *params;                  /* device, layout as in bcf_material */
    uint32_t straight_through;            /* 0 continuous, 1 straight-through */
} bcf_train_material;

/* Device workspace bytes (256-byte aligned start) for the training calls
 * on this material: two texel images of 16 bytes per texel, then 52 MiB +
 * 32 KiB in which the backward sorts its samples by position and keeps
 * dL/d feature per sample (2^20 samples at a time), then the forward's MLP
 * operands in the matrix-core layout (a few KiB). */
bcf_status bcf_train_workspace_size(const bcf_train_material *m, size_t *ws_bytes);

/* G(u, v, s) for n queries (device [n][3]) into out (device [n][dims[n_layers]]),
 * evaluated from the current parameters. At most 2^25 queries per call
 * (BCF_ERR_UNSUPPORTED beyond); n == 0 is a no-op. */
bcf_status bcf_train_forward(const bcf_train_material *m, void *ws, const float *queries, size_t n,
                             float *out, void *stream);

/* Vector-Jacobian product of bcf_train_forward: given grad_out = dL/dG
 * (device [n][dims[n_layers]]), overwrites grad_endpoints[i] (device,
 * texture i's endpoint layout), grad_indices[i] and grad_params (device, the
 * params layout) with dL/d parameter. grad_endpoints and grad_indices are host
 * arrays of n_textures device pointers. Sums use float atomics, so results
 * vary in the last bits from run to run. At most 2^25 queries per call
 * (BCF_ERR_UNSUPPORTED beyond). */
bcf_status bcf_train_backward(const bcf_train_material *m, void *ws, const float *queries, size_t n,
                              const float *grad_out, float *const *grad_endpoints,
                              float *const *grad_indices, float *grad_params, void *stream);

#ifdef __cplusplus
}
#endif
#endif
