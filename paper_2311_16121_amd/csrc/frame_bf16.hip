// Decode kernels with the bf16 MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_bf16(const FrameArgs &a, const MlpShape &sh, bool shared, hipStream_t s)
{
    return shared ? launch_frame_kind<MLP_MFMA_BF16, 16, true>(a, sh, s)
                  : launch_frame_kind<MLP_MFMA_BF16, 16, false>(a, sh, s);
}

}  // namespace bcf
