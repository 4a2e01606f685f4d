// Decode kernels with the fp16 MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_f16(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_frame_kind<MLP_MFMA_F16, 16, kLayoutPacked>(a, sh, s);
    case kLayoutShared: return launch_frame_kind<MLP_MFMA_F16, 16, kLayoutShared>(a, sh, s);
    default: return launch_frame_kind<MLP_MFMA_F16, 16, kLayoutSplit>(a, sh, s);
    }
}

hipError_t launch_batch_f16(const BatchArgs &a, const MlpShape &sh, unsigned grid, uint32_t waves, hipStream_t s)
{
    return launch_batch_kind<MLP_MFMA_F16, 16>(a, sh, grid, waves, s);
}

}  // namespace bcf
