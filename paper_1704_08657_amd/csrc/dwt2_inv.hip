// Kernels and launch of one direction (kInverse); see dwt2_kernels.inl.
#include "dwt2_launch.inl"

namespace dwt2 {

hipError_t launch_inv(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    return kern::launch_dir<kInverse>(wav, dt, sch, cfg, p, planes, s);
}

}  // namespace dwt2
