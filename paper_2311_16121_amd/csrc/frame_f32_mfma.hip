// Decode kernels with the fp32 MFMA MFMA MLP.
#include "frame_kernels.hpp"

namespace bcf {

hipError_t launch_frame_f32_mfma(const FrameArgs &a, const MlpShape &sh, bool shared, hipStream_t s)
{
    return shared ? launch_frame_kind<MLP_MFMA_F32, 16, true>(a, sh, s)
                  : launch_frame_kind<MLP_MFMA_F32, 16, false>(a, sh, s);
}

}  // namespace bcf
