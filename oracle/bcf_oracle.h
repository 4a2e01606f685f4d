/*
 * bcf_oracle.h -- plain CPU oracle for block-compressed neural material decode
 * (Weinreich et al., "Real-Time Neural Materials using Block-Compressed
 * Features", arXiv 2311.16121).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only callers. Nothing on the product
 * path loads this library, and this library shares no code, header, table or
 * constant with the product path.
 *
 * All pointers are host pointers. All arithmetic after the integer BC6H decode
 * is IEEE binary64.
 */
#ifndef BCF_ORACLE_H
#define BCF_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One feature pyramid T_theta_i (Section "Hardware compliant filtering").
 * `blocks` holds levels 0..levels-1 back to back; each level is a row-major
 * grid of 16-byte BC6H blocks covering max(width>>l,1) x max(height>>l,1)
 * texels (a level smaller than 4x4 is one block whose top-left texels are
 * used). `lod_bias` is b_i of the runtime LOD rule (eq. 10). */
typedef struct {
    const uint8_t *blocks;
    uint32_t width, height, levels;
    double lod_bias;
} bcfo_texture;

/* The decoder MLP f_eta (eq. 3): n_layers linear layers with dims[0..n_layers];
 * params holds, per layer, W[dims[l+1]][dims[l]] row-major then b[dims[l+1]]
 * as binary32 values. ReLU after every layer except the last. */
typedef struct {
    uint32_t n_textures;
    const bcfo_texture *textures;
    uint32_t n_layers;
    const uint32_t *dims;
    const float *params;
    int is_signed;              /* 0: BC6H_UF16, 1: BC6H_SF16 */
} bcfo_material;

/* IEEE 754 binary16 bit pattern -> value. */
double bcfo_half_to_double(uint16_t h);

/* Decode one 16-byte BC6H block to 16 texels x (r,g,b) half bit patterns,
 * texel t at (x = t & 3, y = t >> 2). Reserved mode codes give all zeros.
 * Returns the 1-based mode number, or 0 for a reserved code. */
int bcfo_decode_block(const uint8_t block[16], int is_signed, uint16_t out[48]);

/* n blocks -> out[n][16][3]. */
void bcfo_decode_blocks(const uint8_t *blocks, size_t n, int is_signed, uint16_t *out);

/* Header fields of one block as the format definition names them: fields[0..3]
 * = endpoints w, x, y, z (r, g, b each, as stored, before any transform),
 * then partition, mode. Used by tests that inspect the layout. */
int bcfo_block_fields(const uint8_t block[16], int32_t fields[14]);

/* Two-subset partition k (0..31): mask bit t set puts texel t in subset 1;
 * anchor is subset 1's anchor texel. Returns -1 for k out of range. */
int bcfo_partition(int k, uint16_t *mask, int *anchor);

/* Bit budget of a 1-based mode: endpoint/mode/partition bits and index bits.
 * Returns their sum (128 for every valid mode), or -1 for an invalid mode. */
int bcfo_mode_bit_budget(int mode, int *header_bits, int *index_bits);

/* Bytes of a full level chain of `levels` levels for a width x height texture. */
size_t bcfo_texture_bytes(uint32_t width, uint32_t height, uint32_t levels);

/* Trilinear sample T_i(u,v,s) of every texture of the material (eq. 9 with the
 * per-texture LOD of eq. 10), concatenated: feats[n][3*n_textures]. */
void bcfo_sample(const bcfo_material *m, const float *queries, size_t n,
                 double *feats, int n_threads);

/* f_eta applied to z[n][dims[0]] -> out[n][dims[n_layers]]. */
void bcfo_mlp(const bcfo_material *m, const double *z, size_t n, double *out);

/* The whole decode G(u,v,s) (eq. 3): queries[n][3] = (u, v, s) as binary32,
 * out[n][dims[n_layers]]. Work is split over n_threads threads (0 = 1). */
void bcfo_decode(const bcfo_material *m, const float *queries, size_t n,
                 double *out, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
