// Plain fp32 decode kernels (vector ALU MLP).
#include "frame_kernels.hpp"

namespace bcf {

template <int L>
static hipError_t launch_f32_layout(const FrameArgs &a, const MlpShape &sh, hipStream_t s)
{
    return sh.out <= 10 ? launch_frame_kind<MLP_VALU_F32, 10, L>(a, sh, s)
                        : launch_frame_kind<MLP_VALU_F32, 16, L>(a, sh, s);
}

hipError_t launch_frame_f32(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_f32_layout<kLayoutPacked>(a, sh, s);
    case kLayoutShared: return launch_f32_layout<kLayoutShared>(a, sh, s);
    default: return launch_f32_layout<kLayoutSplit>(a, sh, s);
    }
}

hipError_t launch_batch_f32(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s)
{
    return sh.out <= 10 ? launch_batch_kind<MLP_VALU_F32, 10>(a, sh, grid, waves, s)
                        : launch_batch_kind<MLP_VALU_F32, 16>(a, sh, grid, waves, s);
}

}  // namespace bcf
