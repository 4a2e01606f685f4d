// Plain fp32 decode kernels (vector ALU MLP).
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_f32(const FrameArgs &a, const MlpShape &sh, bool shared, hipStream_t s)
{
    if (shared)
        return sh.out <= 10 ? launch_frame_kind<MLP_VALU_F32, 10, true>(a, sh, s)
                            : launch_frame_kind<MLP_VALU_F32, 16, true>(a, sh, s);
    return sh.out <= 10 ? launch_frame_kind<MLP_VALU_F32, 10, false>(a, sh, s)
                        : launch_frame_kind<MLP_VALU_F32, 16, false>(a, sh, s);
}

hipError_t launch_batch_f32(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s)
{
    return sh.out <= 10 ? launch_batch_kind<MLP_VALU_F32, 10>(a, sh, grid, waves, s)
                        : launch_batch_kind<MLP_VALU_F32, 16>(a, sh, grid, waves, s);
}

}  // namespace bcf
