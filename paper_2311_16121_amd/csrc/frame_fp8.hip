// Decode kernels with the fp8 (OCP e4m3) MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_fp8(const FrameArgs &a, const MlpShape &sh, int layout, hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_frame_kind<MLP_MFMA_FP8, 16, kLayoutPacked>(a, sh, s);
    case kLayoutShared: return launch_frame_kind<MLP_MFMA_FP8, 16, kLayoutShared>(a, sh, s);
    default: return launch_frame_kind<MLP_MFMA_FP8, 16, kLayoutSplit>(a, sh, s);
    }
}

}  // namespace bcf
