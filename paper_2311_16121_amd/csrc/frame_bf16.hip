// Decode kernels with the bf16 MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_bf16(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_frame_kind<MLP_MFMA_BF16, 16, kLayoutPacked>(a, sh, s);
    case kLayoutShared: return launch_frame_kind<MLP_MFMA_BF16, 16, kLayoutShared>(a, sh, s);
    default: return launch_frame_kind<MLP_MFMA_BF16, 16, kLayoutSplit>(a, sh, s);
    }
}

}  // namespace bcf
