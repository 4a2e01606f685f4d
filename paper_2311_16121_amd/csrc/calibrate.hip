// The fp8 calibration kernel: the plain fp32 decode recording each layer's
// largest input magnitude.
#include "frame_kernels.hpp"

namespace bcf {

template <int C, int SH>
static hipError_t launch_calib_c(const FrameArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s)
{
#define BCF_CASE(H, NH)                                                                       \
    if (sh.hidden == H && sh.n_hidden == NH) {                                               \
        k_calibrate<H, NH, C, SH><<<grid, kFrameThreads, 0, s>>>(a);                          \
        return hipGetLastError();                                                             \
    }
    BCF_CASE(16, 1) BCF_CASE(16, 2) BCF_CASE(16, 3)
    BCF_CASE(32, 1) BCF_CASE(32, 2) BCF_CASE(32, 3)
    BCF_CASE(64, 1) BCF_CASE(64, 2) BCF_CASE(64, 3)
#undef BCF_CASE
    return hipErrorInvalidValue;
}

template <int L>
static hipError_t launch_calib_layout(const FrameArgs &a, const MlpShape &sh, unsigned grid, hipStream_t s)
{
    return sh.out <= 10 ? launch_calib_c<10, L>(a, sh, grid, s) : launch_calib_c<16, L>(a, sh, grid, s);
}

hipError_t launch_calibrate_kernel(const FrameArgs &a, const MlpShape &sh, int layout, unsigned grid,
                                   hipStream_t s)
{
    switch (layout) {
    case kLayoutPacked: return launch_calib_layout<kLayoutPacked>(a, sh, grid, s);
    case kLayoutShared: return launch_calib_layout<kLayoutShared>(a, sh, grid, s);
    default: return launch_calib_layout<kLayoutSplit>(a, sh, grid, s);
    }
}

}  // namespace bcf
