// Decode kernels with the fp8 (OCP e4m3) MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_fp8(const FrameArgs &a, const MlpShape &sh, bool shared, hipStream_t s)
{
    return shared ? launch_frame_kind<MLP_MFMA_FP8, 16, true>(a, sh, s)
                  : launch_frame_kind<MLP_MFMA_FP8, 16, false>(a, sh, s);
}

}  // namespace bcf
