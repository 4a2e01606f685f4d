// Decode kernels with the fp32 MFMA MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_f32_mfma(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_frame_kind<MLP_MFMA_F32, 16, kLayoutPacked>(a, sh, s);
    case kLayoutShared: return launch_frame_kind<MLP_MFMA_F32, 16, kLayoutShared>(a, sh, s);
    default: return launch_frame_kind<MLP_MFMA_F32, 16, kLayoutSplit>(a, sh, s);
    }
}

}  // namespace bcf
