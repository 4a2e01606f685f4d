// C ABI of the decoder (include/bcf.h): argument validation, workspace layout
// and kernel dispatch. Every launch goes to the caller's stream; nothing here
// synchronises or allocates device memory.
#include "bcf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "train.hpp"

namespace {

thread_local std::string g_error;

bcf_status fail(bcf_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

bcf_status device_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return BCF_OK;
    return fail(BCF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

uint32_t log2u(uint32_t v)
{
    uint32_t r = 0;
    while (v > 1) { v >>= 1; ++r; }
    return r;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

uint32_t level_dim(uint32_t d, uint32_t l) { return (d >> l) ? (d >> l) : 1u; }

// texels per row of a level in the texel scratch (the kernels' row_pitch)
uint32_t scratch_pitch(uint32_t w) { return w + 2u; }

// the texel scratch must stay addressable with 32-bit byte offsets
constexpr size_t kMaxScratchTexels = ((size_t)1 << 31) / 8;

size_t chain_blocks(uint32_t w, uint32_t h, uint32_t levels, uint32_t *per_level_offset)
{
    size_t total = 0;
    for (uint32_t l = 0; l < levels; ++l) {
        if (per_level_offset) per_level_offset[l] = (uint32_t)total;
        total += (size_t)((level_dim(w, l) + 3) / 4) * ((level_dim(h, l) + 3) / 4);
    }
    return total;
}

bool kind_of(bcf_precision p, bcf::MlpKind *k)
{
    switch (p) {
    case BCF_FP32: *k = bcf::MLP_VALU_F32; return true;
    case BCF_FP16: *k = bcf::MLP_MFMA_F16; return true;
    case BCF_BF16: *k = bcf::MLP_MFMA_BF16; return true;
    case BCF_FP8: *k = bcf::MLP_MFMA_FP8; return true;
    case BCF_FP32_MFMA: *k = bcf::MLP_MFMA_F32; return true;
    default: return false;
    }
}

// Validates the material; fills the kernel descriptors and the padded shape.
bcf_status describe(const bcf_material *m, bcf::MaterialDesc *d, bcf::MlpShape *sh)
{
    if (!m) return fail(BCF_ERR_INVALID_ARG, "material is NULL");
    if (m->n_textures < 1 || m->n_textures > (uint32_t)bcf::kMaxTextures)
        return fail(BCF_ERR_INVALID_ARG, "n_textures = %u, expected 1..%d", m->n_textures, bcf::kMaxTextures);
    if (!m->textures) return fail(BCF_ERR_INVALID_ARG, "textures is NULL");
    if (m->is_signed > 1) return fail(BCF_ERR_INVALID_ARG, "is_signed = %u, expected 0 or 1", m->is_signed);
    std::memset(d, 0, sizeof *d);
    d->n_tex = m->n_textures;
    d->is_signed = m->is_signed;
    size_t texel_off = 0;
    for (uint32_t t = 0; t < m->n_textures; ++t) {
        const bcf_texture &x = m->textures[t];
        if (!x.blocks) return fail(BCF_ERR_INVALID_ARG, "texture %u: blocks is NULL", t);
        if (!aligned(x.blocks, 16)) return fail(BCF_ERR_INVALID_ARG, "texture %u: blocks not 16-byte aligned", t);
        if (!is_pow2(x.width) || !is_pow2(x.height) || x.width > 32768 || x.height > 32768)
            return fail(BCF_ERR_INVALID_ARG, "texture %u: %ux%u is not a power-of-two size <= 32768",
                        t, x.width, x.height);
        const uint32_t max_levels = log2u(x.width > x.height ? x.width : x.height) + 1;
        if (x.levels < 1 || x.levels > max_levels)
            return fail(BCF_ERR_INVALID_ARG, "texture %u: levels = %u, expected 1..%u", t, x.levels, max_levels);
        if (!std::isfinite(x.lod_bias)) return fail(BCF_ERR_INVALID_ARG, "texture %u: lod_bias not finite", t);
        bcf::TexDesc &T = d->tex[t];
        T.blocks = static_cast<const uint4 *>(x.blocks);
        T.w = x.width;
        T.h = x.height;
        T.levels = x.levels;
        T.bias = x.lod_bias;
        chain_blocks(x.width, x.height, x.levels, T.blk_off);
        for (uint32_t l = 0; l < x.levels; ++l) {
            T.tex_off[l] = (uint32_t)texel_off;
            texel_off = align_up(texel_off + (size_t)scratch_pitch(level_dim(x.width, l)) * level_dim(x.height, l), 4);
        }
        if (texel_off > kMaxScratchTexels)
            return fail(BCF_ERR_UNSUPPORTED, "material too large: %zu decoded texels, limit %zu",
                        texel_off, kMaxScratchTexels);
    }
    if (m->n_layers < 2 || m->n_layers > 4)
        return fail(BCF_ERR_UNSUPPORTED, "n_layers = %u, supported 2..4 (1..3 hidden layers)", m->n_layers);
    if (!m->dims) return fail(BCF_ERR_INVALID_ARG, "dims is NULL");
    if (!m->params) return fail(BCF_ERR_INVALID_ARG, "params is NULL");
    if (!aligned(m->params, 4)) return fail(BCF_ERR_INVALID_ARG, "params not 4-byte aligned");
    if (m->dims[0] != 3 * m->n_textures)
        return fail(BCF_ERR_INVALID_ARG, "dims[0] = %u, expected 3 * n_textures = %u", m->dims[0], 3 * m->n_textures);
    uint32_t widest = 0;
    for (uint32_t l = 1; l < m->n_layers; ++l) {
        if (m->dims[l] < 1 || m->dims[l] > (uint32_t)bcf::kMaxHidden)
            return fail(BCF_ERR_UNSUPPORTED, "dims[%u] = %u, hidden sizes must be 1..%d", l, m->dims[l], bcf::kMaxHidden);
        widest = m->dims[l] > widest ? m->dims[l] : widest;
    }
    const uint32_t out = m->dims[m->n_layers];
    if (out < 1 || out > (uint32_t)bcf::kMaxOut)
        return fail(BCF_ERR_UNSUPPORTED, "output size %u, supported 1..%d", out, bcf::kMaxOut);
    std::memset(sh, 0, sizeof *sh);
    sh->n_layers = m->n_layers;
    sh->n_hidden = m->n_layers - 1;
    sh->hidden = widest <= 16 ? 16 : widest <= 32 ? 32 : 64;
    sh->out = out;
    for (uint32_t l = 0; l <= m->n_layers; ++l) sh->dims[l] = m->dims[l];
    return BCF_OK;
}

// ---------------------------------------------------------------------------
// Workspace tags. bcf_prepare / bcf_prepare_batch record, per workspace
// address, the precision and a hash of what the workspace was laid out for
// (pyramid geometry and block addresses, MLP shape and parameter address,
// the fp8 activation ranges' address); later calls on that workspace compare
// against the record on the host, so a mismatch is an argument error found
// without reading device memory. The same tag is written into the
// workspace's header.

constexpr uint64_t kFnvOffset = 1469598103934665603ull, kFnvPrime = 1099511628211ull;

uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const uint8_t *b = static_cast<const uint8_t *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * kFnvPrime;
    return h;
}

template <typename T> uint64_t fnv_val(uint64_t h, T v) { return fnv(h, &v, sizeof v); }

// a material that describe() accepted
uint64_t material_hash(uint64_t h, const bcf_material *m, bcf_precision p)
{
    h = fnv_val(h, m->n_textures);
    h = fnv_val(h, m->is_signed);
    for (uint32_t t = 0; t < m->n_textures; ++t) {
        const bcf_texture &x = m->textures[t];
        h = fnv_val(h, reinterpret_cast<uintptr_t>(x.blocks));
        h = fnv_val(h, x.width);
        h = fnv_val(h, x.height);
        h = fnv_val(h, x.levels);
        h = fnv_val(h, x.lod_bias);
    }
    h = fnv_val(h, m->n_layers);
    h = fnv(h, m->dims, sizeof(uint32_t) * (m->n_layers + 1));
    h = fnv_val(h, reinterpret_cast<uintptr_t>(m->params));
    if (p == BCF_FP8) h = fnv_val(h, reinterpret_cast<uintptr_t>(m->act_absmax));
    return h;
}

struct WsTag {
    int precision;
    uint32_t n_materials;
    uint64_t hash;
};

std::mutex g_tags_mu;
std::unordered_map<uintptr_t, WsTag> g_tags;

void remember_ws(const void *ws, const WsTag &tag)
{
    std::lock_guard<std::mutex> lock(g_tags_mu);
    g_tags[reinterpret_cast<uintptr_t>(ws)] = tag;
}

// precision < 0: any precision
bcf_status check_ws(const void *ws, int precision, uint32_t n_materials, uint64_t hash, const char *prepared_by)
{
    WsTag tag;
    {
        std::lock_guard<std::mutex> lock(g_tags_mu);
        const auto it = g_tags.find(reinterpret_cast<uintptr_t>(ws));
        if (it == g_tags.end())
            return fail(BCF_ERR_INVALID_ARG, "workspace %p was not filled by %s", ws, prepared_by);
        tag = it->second;
    }
    if (tag.n_materials != n_materials || tag.hash != hash)
        return fail(BCF_ERR_INVALID_ARG,
                    "workspace %p was prepared for another material (or batch): prepare it again for this one", ws);
    if (precision >= 0 && tag.precision != precision)
        return fail(BCF_ERR_INVALID_ARG, "workspace %p was prepared for precision %d, called with %d", ws,
                    tag.precision, precision);
    return BCF_OK;
}

bcf::WsHeader ws_header(int precision, uint32_t n_materials, uint64_t hash, size_t scratch_off,
                        size_t scratch_bytes, size_t total)
{
    bcf::WsHeader h;
    std::memset(&h, 0, sizeof h);
    h.magic = bcf::kWsMagic;
    h.abi_version = BCF_ABI_VERSION;
    h.precision = (uint32_t)precision;
    h.n_materials = n_materials;
    h.layout_hash = hash;
    h.scratch_off = scratch_off;
    h.scratch_bytes = scratch_bytes;
    h.total_bytes = total;
    return h;
}

// 8-byte units of a material's texel scratch
size_t scratch_texels(const bcf::MaterialDesc &d)
{
    const bcf::TexDesc &T = d.tex[d.n_tex - 1];
    const uint32_t l = T.levels - 1;
    const size_t end = align_up(T.tex_off[l] + (size_t)scratch_pitch(level_dim(T.w, l)) * level_dim(T.h, l), 4);
    return d.interleaved ? end * 3 : end;          // a packed position is three 8-byte units
}

// Switch a material whose four pyramids share one geometry to the
// position-packed scratch (MaterialDesc::interleaved); others keep the
// per-pyramid layout.
void interleave_if_shared(bcf::MaterialDesc &d)
{
    if (d.n_tex != (uint32_t)bcf::kMaxTextures) return;
    const bcf::TexDesc &A = d.tex[0];
    for (uint32_t t = 1; t < d.n_tex; ++t) {
        const bcf::TexDesc &B = d.tex[t];
        if (A.w != B.w || A.h != B.h || A.levels != B.levels || A.bias != B.bias) return;
    }
    size_t pos = 0;
    uint32_t off[bcf::kMaxLevels];
    for (uint32_t l = 0; l < A.levels; ++l) {
        off[l] = (uint32_t)pos;
        pos = align_up(pos + (size_t)scratch_pitch(level_dim(A.w, l)) * level_dim(A.h, l), 4);
    }
    if (pos * 3 > kMaxScratchTexels) return;
    for (uint32_t t = 0; t < d.n_tex; ++t)
        for (uint32_t l = 0; l < A.levels; ++l) d.tex[t].tex_off[l] = off[l];
    d.interleaved = 1;
}

// describe() for the single-material calls: four pyramids of one geometry
// get the packed scratch.
bcf_status describe_single(const bcf_material *m, bcf::MaterialDesc *d, bcf::MlpShape *sh)
{
    const bcf_status st = describe(m, d, sh);
    if (st == BCF_OK) interleave_if_shared(*d);
    return st;
}

size_t elem_bytes(bcf::MlpKind k)
{
    return (k == bcf::MLP_MFMA_F16 || k == bcf::MLP_MFMA_BF16) ? 2 : k == bcf::MLP_MFMA_FP8 ? 1 : 4;
}

// Workspace: a 256-byte header, the texel scratch (at the same offset for
// every precision, so bcf_unpack needs none), then each layer's operands and
// fp32 bias, and the scales.
// MLP operands of precision k from byte offset `base`: each layer's operands
// and fp32 bias, then the scales.
bcf::WsLayout weights_layout(const bcf::MlpShape &sh, bcf::MlpKind k, size_t base)
{
    bcf::WsLayout lay;
    std::memset(&lay, 0, sizeof lay);
    size_t off = base;
    lay.weights_off = off;
    const uint32_t L = sh.n_hidden + 1;
    for (uint32_t l = 0; l < L; ++l) {
        lay.layer_w_off[l] = off;
        off = align_up(off + bcf::mlp_layer_elems(sh, l, k) * elem_bytes(k), 256);
        lay.layer_b_off[l] = off;
        off = align_up(off + (size_t)bcf::mlp_layer_rows(sh, l, k) * 4, 256);
    }
    lay.scales_off = off;
    off = align_up(off + 32 * sizeof(float), 256);
    lay.weights_bytes = off - lay.weights_off;
    lay.total = off;
    return lay;
}

bcf::WsLayout layout(const bcf::MaterialDesc &d, const bcf::MlpShape &sh, bcf::MlpKind k)
{
    const size_t scratch_bytes = scratch_texels(d) * 8;
    bcf::WsLayout lay = weights_layout(sh, k, align_up(256 + scratch_bytes, 256));
    lay.scratch_off = 256;
    lay.scratch_bytes = scratch_bytes;
    return lay;
}

bcf::PredecodePlan predecode_plan(const bcf::MaterialDesc &d)
{
    bcf::PredecodePlan p;
    std::memset(&p, 0, sizeof p);
    uint32_t wg = 0;
    for (uint32_t t = 0; t < (d.interleaved ? 1u : d.n_tex); ++t)
        for (uint32_t l = 0; l < d.tex[t].levels; ++l) {
            uint32_t nb = (uint32_t)(((level_dim(d.tex[t].w, l) + 3) / 4) * ((level_dim(d.tex[t].h, l) + 3) / 4));
            if (d.interleaved) nb *= bcf::kMaxTextures;        // one lane per (block, pyramid)
            p.seg_tex[p.n_seg] = t;
            p.seg_lvl[p.n_seg] = l;
            p.seg_wg[p.n_seg] = wg;
            wg += (nb + 255) / 256;
            ++p.n_seg;
        }
    p.seg_wg[p.n_seg] = wg;
    return p;
}

// The checks shared by bcf_decode and bcf_decode_unpacked.
bcf_status decode_args(const bcf_material *m, bcf_precision p, const void *ws, const float *queries, size_t n,
                       float *out, bcf::MaterialDesc *d, bcf::MlpShape *sh, bcf::MlpKind *kind)
{
    bcf_status st = describe_single(m, d, sh);
    if (st != BCF_OK) return st;
    if (!kind_of(p, kind)) return fail(BCF_ERR_UNSUPPORTED, "precision %d not supported", (int)p);
    if (n == 0) return BCF_OK;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    if (!queries || !aligned(queries, 4)) return fail(BCF_ERR_INVALID_ARG, "queries NULL or misaligned");
    if (!out || !aligned(out, 4)) return fail(BCF_ERR_INVALID_ARG, "out NULL or misaligned");
    if (n > (size_t)1 << 40) return fail(BCF_ERR_UNSUPPORTED, "n = %zu too large", n);
    return check_ws(ws, (int)p, 1u, material_hash(kFnvOffset, m, p), "bcf_prepare");
}

uint2 *scratch_of(void *ws, const bcf::WsLayout &lay)
{
    return reinterpret_cast<uint2 *>(static_cast<uint8_t *>(ws) + lay.scratch_off);
}

bcf_status unpack(const bcf::MaterialDesc &d, const bcf::WsLayout &lay, void *ws, hipStream_t s)
{
    return device_status(bcf::launch_predecode(d, predecode_plan(d), scratch_of(ws, lay), s), "unpack launch");
}


// Validates a trainable material and fills the kernels' descriptor (without
// workspace or gradient pointers). *ws_bytes receives the workspace size.
bcf_status describe_train(const bcf_train_material *m, bcf::TrainDesc *d, size_t *ws_bytes)
{
    if (!m) return fail(BCF_ERR_INVALID_ARG, "material is NULL");
    if (m->n_textures < 1 || m->n_textures > (uint32_t)bcf::kMaxTextures)
        return fail(BCF_ERR_INVALID_ARG, "n_textures = %u, expected 1..%d", m->n_textures, bcf::kMaxTextures);
    if (!m->textures) return fail(BCF_ERR_INVALID_ARG, "textures is NULL");
    if (m->straight_through > 1) return fail(BCF_ERR_INVALID_ARG, "straight_through = %u, expected 0 or 1",
                                             m->straight_through);
    std::memset(d, 0, sizeof *d);
    d->n_tex = m->n_textures;
    d->ste = m->straight_through;
    size_t texels = 0, blocks = 0;
    for (uint32_t t = 0; t < m->n_textures; ++t) {
        const bcf_train_texture &x = m->textures[t];
        if (!is_pow2(x.width) || !is_pow2(x.height) || x.width > 32768 || x.height > 32768)
            return fail(BCF_ERR_INVALID_ARG, "texture %u: %ux%u is not a power-of-two size <= 32768", t, x.width,
                        x.height);
        if (x.levels < 1 || x.levels > log2u(x.width > x.height ? x.width : x.height) + 1)
            return fail(BCF_ERR_INVALID_ARG, "texture %u: levels = %u out of range", t, x.levels);
        if (!std::isfinite(x.lod_bias)) return fail(BCF_ERR_INVALID_ARG, "texture %u: lod_bias not finite", t);
        if (!x.endpoints || !aligned(x.endpoints, 4) || !x.indices || !aligned(x.indices, 4) || !x.partitions)
            return fail(BCF_ERR_INVALID_ARG, "texture %u: endpoints, indices or partitions NULL or misaligned", t);
        bcf::TrainTexDesc &td = d->tex[t];
        td.endpoints = x.endpoints;
        td.indices = x.indices;
        td.partitions = x.partitions;
        td.w = x.width;
        td.h = x.height;
        td.levels = x.levels;
        td.bias = x.lod_bias;
        td.n_blocks = (uint32_t)chain_blocks(x.width, x.height, x.levels, td.blk_off);
        d->blk_base[t] = (uint32_t)blocks;
        blocks += td.n_blocks;
        for (uint32_t l = 0; l < x.levels; ++l) {
            td.tex_off[l] = (uint32_t)texels;
            texels += (size_t)level_dim(x.width, l) * level_dim(x.height, l);
        }
    }
    d->blk_base[m->n_textures] = (uint32_t)blocks;
    if (texels > ((size_t)1 << 27)) return fail(BCF_ERR_UNSUPPORTED, "%zu texels, at most 2^27", texels);
    d->n_texels = (uint32_t)texels;
    if (m->n_layers < 2 || m->n_layers > 4)
        return fail(BCF_ERR_UNSUPPORTED, "n_layers = %u, expected 2..4", m->n_layers);
    if (!m->dims) return fail(BCF_ERR_INVALID_ARG, "dims is NULL");
    if (m->dims[0] != 3 * m->n_textures)
        return fail(BCF_ERR_INVALID_ARG, "dims[0] = %u, expected 3 * n_textures = %u", m->dims[0], 3 * m->n_textures);
    const uint32_t hidden = m->dims[1];
    for (uint32_t l = 1; l < m->n_layers; ++l)
        if (m->dims[l] != hidden || (hidden != 16 && hidden != 32))
            return fail(BCF_ERR_UNSUPPORTED, "hidden widths must all be 16 or 32 for training (dims[%u] = %u)", l,
                        m->dims[l]);
    const uint32_t out = m->dims[m->n_layers];
    if (out < 1 || out > (uint32_t)bcf::kMaxOut)
        return fail(BCF_ERR_UNSUPPORTED, "output width %u, expected 1..%d", out, bcf::kMaxOut);
    if (!m->params || !aligned(m->params, 4)) return fail(BCF_ERR_INVALID_ARG, "params NULL or misaligned");
    d->params = m->params;
    d->n_layers = m->n_layers;
    uint32_t off = 0;
    for (uint32_t l = 0; l < m->n_layers; ++l) {
        d->dims[l] = m->dims[l];
        d->w_off[l] = off;
        off += m->dims[l] * m->dims[l + 1];
        d->b_off[l] = off;
        off += m->dims[l + 1];
    }
    d->dims[m->n_layers] = out;
    d->n_params = off;
    bcf::MlpShape &sh = d->ops_shape;
    sh.n_layers = m->n_layers;
    sh.n_hidden = m->n_layers - 1;
    sh.hidden = hidden;
    sh.out = out;
    for (uint32_t l = 0; l <= m->n_layers; ++l) sh.dims[l] = m->dims[l];
    const size_t sort_end = 2 * align_up(texels * 16, 256) + align_up((size_t)bcf::kTrainBinBatch * 4, 256) +
                            2 * align_up((size_t)bcf::kTrainBins * 4, 256) + (size_t)bcf::kTrainBinBatch * 48;
    d->ops = weights_layout(sh, bcf::MLP_MFMA_F32, align_up(sort_end, 256));
    *ws_bytes = d->ops.total;
    return BCF_OK;
}

// The workspace holds bcf_train_workspace_size bytes (the caller's promise):
// the texel values, their gradients, then the backward's sample sort.
bcf_status bind_train_ws(bcf::TrainDesc *d, void *ws)
{
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    uint8_t *p = static_cast<uint8_t *>(ws);
    const size_t img = align_up((size_t)d->n_texels * 16, 256);
    d->texels = reinterpret_cast<float4 *>(p);
    d->g_texels = reinterpret_cast<float4 *>(p + img);
    p += 2 * img;
    d->bin_perm = reinterpret_cast<uint32_t *>(p);
    p += align_up((size_t)bcf::kTrainBinBatch * 4, 256);
    d->bin_count = reinterpret_cast<uint32_t *>(p);
    p += align_up((size_t)bcf::kTrainBins * 4, 256);
    d->bin_next = reinterpret_cast<uint32_t *>(p);
    p += align_up((size_t)bcf::kTrainBins * 4, 256);
    d->bin_dz = reinterpret_cast<float *>(p);
    d->ops_ws = static_cast<uint8_t *>(ws);
    return BCF_OK;
}

// A batch: every material valid, one MLP shape; the workspace holds a 256-byte
// header, the material table, the item prefix, the unpack segment table and
// its chunk map, then per material its texel scratch, then the MLP operands.
struct BatchLayout {
    size_t table_off, items_off, segs_off, chunk_seg_off, marks_off, units_off, total;
    uint32_t n_seg, n_chunks;               // unpack segments of every material, their chunks of 256 lanes
    uint32_t n_units;                       // work units of the touched-blocks unpack
    std::vector<bcf::BatchSlot> slots;
    std::vector<bcf::MaterialDesc> descs;
    bcf::MlpShape sh;
    bcf::WsLayout rel;
    bcf::MlpKind kind;
};

constexpr uint32_t kMaxBatch = 4096;

bcf_status describe_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, BatchLayout *b)
{
    if (!mats) return fail(BCF_ERR_INVALID_ARG, "materials is NULL");
    if (n_mats < 1 || n_mats > kMaxBatch) return fail(BCF_ERR_INVALID_ARG, "n_mats = %u, expected 1..%u", n_mats, kMaxBatch);
    if (!kind_of(p, &b->kind)) return fail(BCF_ERR_UNSUPPORTED, "precision %d not supported", (int)p);
    if (b->kind != bcf::MLP_MFMA_F16 && b->kind != bcf::MLP_VALU_F32)
        return fail(BCF_ERR_UNSUPPORTED, "batched decode runs BCF_FP16 or BCF_FP32");
    b->descs.resize(n_mats);
    b->slots.resize(n_mats);
    size_t off = 256;
    b->table_off = off;
    off = align_up(off + bcf::batch_table_bytes(n_mats), 256);
    b->items_off = off;
    off = align_up(off + (size_t)(n_mats + 1) * 4, 256);
    b->segs_off = off;                      // its size is known once the materials are described
    b->n_seg = 0;
    b->n_chunks = 0;
    b->n_units = 0;
    for (uint32_t k = 0; k < n_mats; ++k) {
        bcf::MlpShape sh;
        const bcf_status st = describe(&mats[k], &b->descs[k], &sh);
        if (st != BCF_OK) {
            const std::string why = g_error;
            return fail(st, "material %u: %s", k, why.c_str());
        }
        if (k == 0) {
            b->sh = sh;
        } else if (sh.n_layers != b->sh.n_layers ||
                   std::memcmp(sh.dims, b->sh.dims, sizeof(uint32_t) * (sh.n_layers + 1)) != 0) {
            return fail(BCF_ERR_INVALID_ARG, "material %u: MLP dims differ from material 0", k);
        }
        interleave_if_shared(b->descs[k]);
        const bcf::PredecodePlan plan = predecode_plan(b->descs[k]);
        b->n_seg += plan.n_seg;
        b->n_chunks += plan.seg_wg[plan.n_seg];
        for (uint32_t j = 0; j < plan.n_seg; ++j) {
            const uint32_t chunks = plan.seg_wg[j + 1] - plan.seg_wg[j];
            b->n_units += b->descs[k].interleaved ? (chunks + 3) / 4 : chunks;
        }
    }
    off = align_up(off + sizeof(bcf::UnpackSeg) * b->n_seg, 256);
    b->chunk_seg_off = off;                 // segment of each unpack chunk
    off = align_up(off + sizeof(uint32_t) * b->n_chunks, 256);
    b->marks_off = off;                     // one byte per block position of every chunk
    off = align_up(off + (size_t)64 * b->n_chunks, 256);
    b->units_off = off;                     // first chunk of each touched-unpack unit
    off = align_up(off + sizeof(uint32_t) * b->n_units, 256);
    for (uint32_t k = 0; k < n_mats; ++k) {
        b->slots[k].scratch_off = off;
        b->slots[k].scratch_bytes = scratch_texels(b->descs[k]) * 8;
        off = align_up(off + b->slots[k].scratch_bytes, 256);
    }
    b->rel = weights_layout(b->sh, b->kind, 0);
    for (uint32_t k = 0; k < n_mats; ++k) {
        b->slots[k].weights_off = off;
        off += b->rel.weights_bytes;
    }
    b->total = off;
    return BCF_OK;
}

uint64_t batch_hash(const bcf_material *mats, uint32_t n_mats, bcf_precision p)
{
    uint64_t h = fnv_val(kFnvOffset, n_mats);
    for (uint32_t k = 0; k < n_mats; ++k) h = material_hash(h, &mats[k], p);
    return h;
}

}  // namespace

extern "C" {

int bcf_abi_version(void) { return BCF_ABI_VERSION; }

const char *bcf_last_error(void) { return g_error.c_str(); }

size_t bcf_texture_bytes(uint32_t width, uint32_t height, uint32_t levels)
{
    if (!is_pow2(width) || !is_pow2(height) || width > 32768 || height > 32768) return 0;
    if (levels < 1 || levels > log2u(width > height ? width : height) + 1) return 0;
    return 16 * chain_blocks(width, height, levels, nullptr);
}

bcf_status bcf_prepare(const bcf_material *m, bcf_precision p, void *ws, size_t *ws_bytes, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf_status st = describe_single(m, &d, &sh);
    if (st != BCF_OK) return st;
    bcf::MlpKind kind;
    if (!kind_of(p, &kind)) return fail(BCF_ERR_UNSUPPORTED, "precision %d not supported", (int)p);
    if (!ws_bytes) return fail(BCF_ERR_INVALID_ARG, "ws_bytes is NULL");
    const bcf::WsLayout lay = layout(d, sh, kind);
    if (!ws) {
        *ws_bytes = lay.total;
        return BCF_OK;
    }
    if (*ws_bytes < lay.total)
        return fail(BCF_ERR_INVALID_ARG, "workspace of %zu bytes, need %zu", *ws_bytes, lay.total);
    if (!aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (kind == bcf::MLP_MFMA_FP8 && !m->act_absmax)
        return fail(BCF_ERR_INVALID_ARG, "BCF_FP8 needs act_absmax (see bcf_calibrate)");
    if (m->act_absmax && !aligned(m->act_absmax, 4))
        return fail(BCF_ERR_INVALID_ARG, "act_absmax not 4-byte aligned");
    const uint64_t hash = material_hash(kFnvOffset, m, p);
    const bcf::WsHeader header = ws_header(p, 1, hash, lay.scratch_off, lay.scratch_bytes, lay.total);
    st = device_status(bcf::launch_prepare_weights(m->params, m->act_absmax, sh, kind, lay, ws, &header,
                                                   static_cast<hipStream_t>(stream)),
                       "prepare launch");
    if (st == BCF_OK) remember_ws(ws, WsTag{(int)p, 1u, hash});
    return st;
}


bcf_status bcf_decode(const bcf_material *m, bcf_precision p, void *ws, const float *queries, size_t n,
                      uint32_t grid_width, float *out, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf::MlpKind kind;
    bcf_status st = decode_args(m, p, ws, queries, n, out, &d, &sh, &kind);
    if (st != BCF_OK || n == 0) return st;
    const bcf::WsLayout lay = layout(d, sh, kind);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = unpack(d, lay, ws, s);
    if (st != BCF_OK) return st;
    return device_status(bcf::launch_filter_mlp(d, sh, kind, lay, ws, queries, n, grid_width, out, s),
                         "decode launch");
}

bcf_status bcf_unpack(const bcf_material *m, void *ws, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf_status st = describe_single(m, &d, &sh);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    // any precision: the scratch sits at the same offset in every precision's layout
    {
        std::lock_guard<std::mutex> lock(g_tags_mu);
        const auto it = g_tags.find(reinterpret_cast<uintptr_t>(ws));
        if (it == g_tags.end())
            return fail(BCF_ERR_INVALID_ARG, "workspace %p was not filled by bcf_prepare", ws);
        if (it->second.n_materials != 1 ||
            it->second.hash != material_hash(kFnvOffset, m, (bcf_precision)it->second.precision))
            return fail(BCF_ERR_INVALID_ARG,
                        "workspace %p was prepared for another material: prepare it again for this one", ws);
    }
    const bcf::WsLayout lay = layout(d, sh, bcf::MLP_VALU_F32);
    return unpack(d, lay, ws, static_cast<hipStream_t>(stream));
}

bcf_status bcf_decode_unpacked(const bcf_material *m, bcf_precision p, const void *ws, const float *queries,
                               size_t n, uint32_t grid_width, float *out, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf::MlpKind kind;
    bcf_status st = decode_args(m, p, ws, queries, n, out, &d, &sh, &kind);
    if (st != BCF_OK || n == 0) return st;
    const bcf::WsLayout lay = layout(d, sh, kind);
    return device_status(bcf::launch_filter_mlp(d, sh, kind, lay, ws, queries, n, grid_width, out,
                                                static_cast<hipStream_t>(stream)),
                         "decode launch");
}

bcf_status bcf_calibrate(const bcf_material *m, void *ws, const float *queries, size_t n,
                         float *act_absmax, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf_status st = describe_single(m, &d, &sh);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    if (!act_absmax || !aligned(act_absmax, 4)) return fail(BCF_ERR_INVALID_ARG, "act_absmax NULL or misaligned");
    if (n > 0 && (!queries || !aligned(queries, 4)))
        return fail(BCF_ERR_INVALID_ARG, "queries NULL or misaligned");
    if ((st = check_ws(ws, BCF_FP32, 1u, material_hash(kFnvOffset, m, BCF_FP32), "bcf_prepare")) != BCF_OK)
        return st;
    const bcf::WsLayout lay = layout(d, sh, bcf::MLP_VALU_F32);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = unpack(d, lay, ws, s);
    if (st != BCF_OK) return st;
    return device_status(bcf::launch_calibrate(d, sh, lay, ws, queries, n, act_absmax, s), "calibrate launch");
}

bcf_status bcf_decode_noalloc(const bcf_material *m, bcf_precision p, const float *queries, size_t n,
                              uint32_t grid_width, float *out, void *stream)
{
    bcf::MaterialDesc d;
    bcf::MlpShape sh;
    bcf::MlpKind kind;
    bcf_status st = describe_single(m, &d, &sh);
    if (st != BCF_OK) return st;
    if (!kind_of(p, &kind)) return fail(BCF_ERR_UNSUPPORTED, "precision %d not supported", (int)p);
    if (n == 0) return BCF_OK;
    if (!queries || !aligned(queries, 4)) return fail(BCF_ERR_INVALID_ARG, "queries NULL or misaligned");
    if (!out || !aligned(out, 4)) return fail(BCF_ERR_INVALID_ARG, "out NULL or misaligned");
    if (n > (size_t)1 << 40) return fail(BCF_ERR_UNSUPPORTED, "n = %zu too large", n);
    if (kind == bcf::MLP_MFMA_FP8 && !m->act_absmax)
        return fail(BCF_ERR_INVALID_ARG, "BCF_FP8 needs act_absmax (see bcf_calibrate)");
    if (m->act_absmax && !aligned(m->act_absmax, 4))
        return fail(BCF_ERR_INVALID_ARG, "act_absmax not 4-byte aligned");
    const bcf::WsLayout lay = layout(d, sh, kind);
    if (lay.total > bcf::kNoAllocBytes)
        return fail(BCF_ERR_UNSUPPORTED,
                    "bcf_decode_noalloc: this material needs a %zu-byte workspace, the library's own holds %zu "
                    "(use bcf_prepare and bcf_decode with a caller workspace)",
                    lay.total, bcf::kNoAllocBytes);
    void *ws = nullptr;
    if ((st = device_status(bcf::noalloc_workspace(&ws), "library workspace lookup")) != BCF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bcf::WsHeader header = ws_header(p, 1, material_hash(kFnvOffset, m, p), lay.scratch_off,
                                           lay.scratch_bytes, lay.total);
    st = device_status(bcf::launch_prepare_weights(m->params, m->act_absmax, sh, kind, lay, ws, &header, s),
                       "prepare launch");
    if (st != BCF_OK) return st;
    if ((st = unpack(d, lay, ws, s)) != BCF_OK) return st;
    return device_status(bcf::launch_filter_mlp(d, sh, kind, lay, ws, queries, n, grid_width, out, s),
                         "decode launch");
}

bcf_status bcf_decode_blocks(const void *blocks, size_t n_blocks, uint32_t is_signed, uint16_t *halves,
                             void *stream)
{
    if (is_signed > 1) return fail(BCF_ERR_INVALID_ARG, "is_signed = %u, expected 0 or 1", is_signed);
    if (n_blocks == 0) return BCF_OK;
    if (!blocks || !aligned(blocks, 16)) return fail(BCF_ERR_INVALID_ARG, "blocks NULL or not 16-byte aligned");
    if (!halves || !aligned(halves, 16)) return fail(BCF_ERR_INVALID_ARG, "halves NULL or not 16-byte aligned");
    return device_status(bcf::launch_decode_blocks(static_cast<const uint4 *>(blocks), n_blocks, is_signed,
                                                   halves, static_cast<hipStream_t>(stream)),
                         "decode_blocks launch");
}

bcf_status bcf_train_workspace_size(const bcf_train_material *m, size_t *ws_bytes)
{
    if (!ws_bytes) return fail(BCF_ERR_INVALID_ARG, "ws_bytes is NULL");
    bcf::TrainDesc d;
    return describe_train(m, &d, ws_bytes);
}

bcf_status bcf_train_forward(const bcf_train_material *m, void *ws, const float *queries, size_t n, float *out,
                             void *stream)
{
    bcf::TrainDesc d;
    size_t need;
    bcf_status st = describe_train(m, &d, &need);
    if (st != BCF_OK) return st;
    if (n == 0) return BCF_OK;
    if ((st = bind_train_ws(&d, ws)) != BCF_OK) return st;
    if (!queries || !aligned(queries, 4)) return fail(BCF_ERR_INVALID_ARG, "queries NULL or misaligned");
    if (!out || !aligned(out, 4)) return fail(BCF_ERR_INVALID_ARG, "out NULL or misaligned");
    if (n > bcf::kMaxQueriesPerLaunch) return fail(BCF_ERR_UNSUPPORTED, "n = %zu, at most 2^25", n);
    return device_status(bcf::launch_train_forward(d, queries, n, out, static_cast<hipStream_t>(stream)),
                         "train forward launch");
}

bcf_status bcf_train_backward(const bcf_train_material *m, void *ws, const float *queries, size_t n,
                              const float *grad_out, float *const *grad_endpoints, float *const *grad_indices,
                              float *grad_params, void *stream)
{
    bcf::TrainDesc d;
    size_t need;
    bcf_status st = describe_train(m, &d, &need);
    if (st != BCF_OK) return st;
    if ((st = bind_train_ws(&d, ws)) != BCF_OK) return st;
    if (n > 0 && (!queries || !aligned(queries, 4) || !grad_out || !aligned(grad_out, 4)))
        return fail(BCF_ERR_INVALID_ARG, "queries or grad_out NULL or misaligned");
    if (n > bcf::kMaxQueriesPerLaunch) return fail(BCF_ERR_UNSUPPORTED, "n = %zu, at most 2^25", n);
    if (!grad_endpoints || !grad_indices) return fail(BCF_ERR_INVALID_ARG, "gradient pointer arrays NULL");
    if (!grad_params || !aligned(grad_params, 4)) return fail(BCF_ERR_INVALID_ARG, "grad_params NULL or misaligned");
    for (uint32_t t = 0; t < d.n_tex; ++t) {
        if (!grad_endpoints[t] || !aligned(grad_endpoints[t], 4) || !grad_indices[t] || !aligned(grad_indices[t], 4))
            return fail(BCF_ERR_INVALID_ARG, "texture %u: gradient buffers NULL or misaligned", t);
        d.tex[t].g_endpoints = grad_endpoints[t];
        d.tex[t].g_indices = grad_indices[t];
    }
    d.g_params = grad_params;
    return device_status(bcf::launch_train_backward(d, queries, n, grad_out, static_cast<hipStream_t>(stream)),
                         "train backward launch");
}

bcf_status bcf_batch_workspace_size(const bcf_material *mats, uint32_t n_mats, bcf_precision p, size_t *ws_bytes)
{
    if (!ws_bytes) return fail(BCF_ERR_INVALID_ARG, "ws_bytes is NULL");
    BatchLayout b;
    const bcf_status st = describe_batch(mats, n_mats, p, &b);
    if (st == BCF_OK) *ws_bytes = b.total;
    return st;
}

bcf_status bcf_prepare_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws, size_t ws_bytes,
                             void *stream)
{
    BatchLayout b;
    bcf_status st = describe_batch(mats, n_mats, p, &b);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < b.total) return fail(BCF_ERR_INVALID_ARG, "workspace of %zu bytes, need %zu", ws_bytes, b.total);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (uint32_t k = 0; k < n_mats; ++k) {
        st = device_status(bcf::launch_prepare_weights(mats[k].params, nullptr, b.sh, b.kind, b.rel,
                                                       static_cast<uint8_t *>(ws) + b.slots[k].weights_off,
                                                       nullptr, s),
                           "prepare launch");
        if (st != BCF_OK) return st;
    }
    // the unpack segments of every material, numbered in one sequence of chunks
    std::vector<bcf::UnpackSeg> segs;
    std::vector<uint32_t> chunk_seg(b.n_chunks), units;
    segs.reserve(b.n_seg);
    units.reserve(b.n_units);
    uint32_t chunk0 = 0;
    for (uint32_t k = 0; k < n_mats; ++k) {
        const bcf::MaterialDesc &d = b.descs[k];
        const bcf::PredecodePlan plan = predecode_plan(d);
        uint2 *texels = reinterpret_cast<uint2 *>(static_cast<uint8_t *>(ws) + b.slots[k].scratch_off);
        for (uint32_t j = 0; j < plan.n_seg; ++j) {
            const uint32_t l = plan.seg_lvl[j];
            const bcf::TexDesc &T0 = d.tex[d.interleaved ? 0u : plan.seg_tex[j]];
            bcf::UnpackSeg g;
            std::memset(&g, 0, sizeof g);
            for (uint32_t t = 0; t < (uint32_t)bcf::kMaxTextures; ++t) {
                const bcf::TexDesc &T = d.interleaved ? d.tex[t < d.n_tex ? t : 0u] : T0;
                g.blocks[t] = T.blocks + T.blk_off[l];
            }
            // 8-byte units per position: 3 packed, 1 per pyramid
            g.texels = texels + (d.interleaved ? 3u : 1u) * (size_t)T0.tex_off[l];
            g.lw = level_dim(T0.w, l);
            g.lh = level_dim(T0.h, l);
            g.wg0 = chunk0 + plan.seg_wg[j];
            g.flags = (d.interleaved ? bcf::kSegInterleaved : 0u) | (d.is_signed ? bcf::kSegSigned : 0u);
            const uint32_t end = chunk0 + plan.seg_wg[j + 1];
            std::fill(chunk_seg.begin() + g.wg0, chunk_seg.begin() + end, (uint32_t)segs.size());
            for (uint32_t c = g.wg0; c < end; c += d.interleaved ? 4u : 1u) units.push_back(c);
            if (d.interleaved) b.slots[k].seg_chunk[l] = g.wg0;
            segs.push_back(g);
        }
        chunk0 += plan.seg_wg[plan.n_seg];
    }
    if (!units.empty()) {
        // write_batch_table below synchronises the stream before `units` goes
        st = device_status(hipMemcpyAsync(static_cast<uint8_t *>(ws) + b.units_off, units.data(),
                                          sizeof(uint32_t) * units.size(), hipMemcpyHostToDevice, s),
                           "unit table copy");
        if (st != BCF_OK) return st;
    }
    const uint64_t hash = batch_hash(mats, n_mats, p);
    st = device_status(bcf::write_batch_table(b.descs.data(), b.slots.data(), n_mats, b.sh.out,
                                              ws_header(p, n_mats, hash, 0, 0, b.total), ws, b.table_off,
                                              segs.data(), (uint32_t)segs.size(), b.segs_off, chunk_seg.data(),
                                              b.n_chunks, b.chunk_seg_off, s),
                       "material table copy");
    if (st == BCF_OK) remember_ws(ws, WsTag{(int)p, n_mats, hash});
    return st;
}

bcf_status bcf_unpack_batch(const bcf_material *mats, uint32_t n_mats, void *ws, void *stream)
{
    BatchLayout b;
    bcf_status st = describe_batch(mats, n_mats, BCF_FP16, &b);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    // either batch precision: the texel scratch layout is the same (and so is the hash)
    if ((st = check_ws(ws, -1, n_mats, batch_hash(mats, n_mats, BCF_FP16), "bcf_prepare_batch")) != BCF_OK)
        return st;
    // one launch over the segment table bcf_prepare_batch wrote
    const uint8_t *base = static_cast<const uint8_t *>(ws);
    const bcf::UnpackSeg *segs = reinterpret_cast<const bcf::UnpackSeg *>(base + b.segs_off);
    const uint32_t *chunk_seg = reinterpret_cast<const uint32_t *>(base + b.chunk_seg_off);
    return device_status(bcf::launch_predecode_batch(segs, chunk_seg, b.n_chunks, static_cast<hipStream_t>(stream)),
                         "unpack launch");
}

namespace {

bcf_status batch_args(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws, const float *queries,
                      const uint32_t *offsets, uint32_t n_total, float *out, BatchLayout *b)
{
    const bcf_status st = describe_batch(mats, n_mats, p, b);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    if (!offsets || !aligned(offsets, 4)) return fail(BCF_ERR_INVALID_ARG, "offsets NULL or misaligned");
    if (n_total > 0 && (!queries || !aligned(queries, 4) || !out || !aligned(out, 4)))
        return fail(BCF_ERR_INVALID_ARG, "queries or out NULL or misaligned");
    return check_ws(ws, (int)p, n_mats, batch_hash(mats, n_mats, p), "bcf_prepare_batch");
}

unsigned default_workgroups(uint32_t n_total)
{
    const uint64_t items = ((uint64_t)n_total + 63) / 64;
    return (unsigned)std::min<uint64_t>(std::max<uint64_t>((items + 3) / 4, 8), 2048);
}

}  // namespace

bcf_status bcf_unpack_batch_touched(const bcf_material *mats, uint32_t n_mats, void *ws, const float *queries,
                                    const uint32_t *offsets, uint32_t n_total, void *stream)
{
    BatchLayout b;
    bcf_status st = describe_batch(mats, n_mats, BCF_FP16, &b);
    if (st != BCF_OK) return st;
    if (!ws || !aligned(ws, 256)) return fail(BCF_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    if (!offsets || !aligned(offsets, 4)) return fail(BCF_ERR_INVALID_ARG, "offsets NULL or misaligned");
    if (n_total > 0 && (!queries || !aligned(queries, 4)))
        return fail(BCF_ERR_INVALID_ARG, "queries NULL or misaligned");
    // either batch precision: the tables and the scratch layout are the same (and so is the hash)
    if ((st = check_ws(ws, -1, n_mats, batch_hash(mats, n_mats, BCF_FP16), "bcf_prepare_batch")) != BCF_OK)
        return st;
    uint8_t *base = static_cast<uint8_t *>(ws);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    st = device_status(bcf::launch_batch_mark(ws, b.table_off, b.items_off, queries, offsets, n_mats, n_total,
                                              base + b.marks_off, (size_t)64 * b.n_chunks, s),
                       "mark launch");
    if (st != BCF_OK) return st;
    return device_status(bcf::launch_predecode_touched(reinterpret_cast<const bcf::UnpackSeg *>(base + b.segs_off),
                                                       reinterpret_cast<const uint32_t *>(base + b.chunk_seg_off),
                                                       b.n_seg, b.n_chunks,
                                                       reinterpret_cast<const uint32_t *>(base + b.units_off),
                                                       b.n_units, base + b.marks_off, s),
                         "unpack launch");
}

bcf_status bcf_decode_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws,
                            const float *queries, const uint32_t *offsets, uint32_t n_total, float *out,
                            const bcf_batch_plan *plan, void *stream)
{
    if (plan && (plan->waves != 0 && plan->waves != 2 && plan->waves != 4))
        return fail(BCF_ERR_INVALID_ARG, "plan->waves = %u, expected 0, 2 or 4", plan->waves);
    if (plan && plan->run > 64) return fail(BCF_ERR_INVALID_ARG, "plan->run = %u, at most 64", plan->run);
    BatchLayout b;
    const bcf_status st = batch_args(mats, n_mats, p, ws, queries, offsets, n_total, out, &b);
    if (st != BCF_OK) return st;
    bcf::BatchShape shape;
    shape.workgroups = plan && plan->workgroups ? plan->workgroups : default_workgroups(n_total);
    shape.interleave = plan ? (plan->interleave ? 1u : 0u) : 1u;
    shape.run = plan && plan->run ? plan->run : 1u;
    shape.waves = plan && plan->waves ? plan->waves : 4u;
    return device_status(bcf::launch_batch(ws, b.table_off, b.items_off, b.rel, b.sh, b.kind, queries, offsets, n_mats,
                                           n_total, out, shape, static_cast<hipStream_t>(stream)),
                         "batch launch");
}

bcf_status bcf_tune_batch(const bcf_material *mats, uint32_t n_mats, bcf_precision p, void *ws,
                          const float *queries, const uint32_t *offsets, uint32_t n_total, float *out,
                          bcf_batch_plan *best, float *best_ms, void *stream)
{
    BatchLayout b;
    bcf_status st = batch_args(mats, n_mats, p, ws, queries, offsets, n_total, out, &b);
    if (st != BCF_OK) return st;
    if (!best) return fail(BCF_ERR_INVALID_ARG, "best is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if ((st = device_status(hipEventCreate(&e0), "event")) != BCF_OK) return st;
    if ((st = device_status(hipEventCreate(&e1), "event")) != BCF_OK) {
        (void)hipEventDestroy(e0);
        return st;
    }
    // candidate shapes: total waves from 1024 to 16384 in 2- or 4-wave
    // workgroups; contiguous ranges, or interleaved runs of 1, 2 or 4 items
    static const unsigned kWaves[] = {1024, 2048, 4096, 8192, 16384};
    static const uint32_t kRuns[] = {0, 1, 2, 4};          // 0: contiguous ranges
    float best_t = -1.0f;
    bcf_batch_plan pick = {default_workgroups(n_total), 1, 1, 4};
    for (unsigned tw : kWaves)
    for (uint32_t waves = 2; waves <= 4 && st == BCF_OK; waves += 2) {
        for (uint32_t r = 0; r < 4 && st == BCF_OK; ++r) {
            const bcf::BatchShape shape{tw / waves, kRuns[r] ? 1u : 0u, kRuns[r] ? kRuns[r] : 1u, waves};
            auto run = [&]() {
                return device_status(bcf::launch_batch(ws, b.table_off, b.items_off, b.rel, b.sh, b.kind, queries,
                                                       offsets, n_mats, n_total, out, shape, s),
                                     "batch launch");
            };
            if ((st = run()) != BCF_OK) break;                       // warm-up
            (void)hipEventRecord(e0, s);
            for (int rep = 0; rep < 3 && st == BCF_OK; ++rep) st = run();
            (void)hipEventRecord(e1, s);
            if (st != BCF_OK || (st = device_status(hipEventSynchronize(e1), "tune sync")) != BCF_OK) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= 3.0f;
            if (best_t < 0.0f || ms < best_t) {
                best_t = ms;
                pick = bcf_batch_plan{shape.workgroups, shape.interleave, shape.run, shape.waves};
            }
        }
        if (st != BCF_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != BCF_OK) return st;
    *best = pick;
    if (best_ms) *best_ms = best_t;
    return BCF_OK;
}

}  // extern "C"
