// Test-only: the GPU library's BC6H unpacking (bc6h_device.hpp), compiled for
// the host so its integer logic can be compared with the oracle on the CPU.
#include <hip/hip_runtime.h>

#include "bc6h_device.hpp"

extern "C" void shim_decode_blocks(const uint32_t *blocks, size_t n, int is_signed, uint16_t *out)
{
    for (size_t i = 0; i < n; ++i) {
        const uint32_t *b = blocks + 4 * i;
        bcf::Bc6hHeader h;
        if (is_signed) bcf::bc6h_header<true>(b[0], b[1], b[2], b[3], bcf::kTable, h);
        else bcf::bc6h_header<false>(b[0], b[1], b[2], b[3], bcf::kTable, h);
        for (uint32_t t = 0; t < 16; ++t)
            for (int c = 0; c < 3; ++c)
                out[48 * i + 3 * t + c] = (uint16_t)(is_signed ? bcf::bc6h_texel<true>(h, t, c)
                                                               : bcf::bc6h_texel<false>(h, t, c));
    }
}

// The same through the palette the unpack kernel uses.
extern "C" void shim_decode_blocks_palette(const uint32_t *blocks, size_t n, int is_signed, uint16_t *out)
{
    for (size_t i = 0; i < n; ++i) {
        const uint32_t *b = blocks + 4 * i;
        bcf::Bc6hHeader h;
        uint32_t pal[16][2];
        if (is_signed) {
            bcf::bc6h_header<true>(b[0], b[1], b[2], b[3], bcf::kTable, h);
            bcf::bc6h_palette<true>(h, pal);
        } else {
            bcf::bc6h_header<false>(b[0], b[1], b[2], b[3], bcf::kTable, h);
            bcf::bc6h_palette<false>(h, pal);
        }
        uint32_t s0, s1;
        bcf::bc6h_slots(h, s0, s1);
        for (uint32_t t = 0; t < 16; ++t) {
            const uint32_t j = ((t < 8 ? s0 : s1) >> (4 * (t & 7))) & 15u;
            if (j != bcf::bc6h_slot(h, t)) {
                out[48 * i + 3 * t] = 0xDEADu;      // the packed slots disagree with the per-texel ones
                continue;
            }
            out[48 * i + 3 * t + 0] = (uint16_t)(pal[j][0] & 0xFFFFu);
            out[48 * i + 3 * t + 1] = (uint16_t)(pal[j][0] >> 16);
            out[48 * i + 3 * t + 2] = (uint16_t)pal[j][1];
        }
    }
}
