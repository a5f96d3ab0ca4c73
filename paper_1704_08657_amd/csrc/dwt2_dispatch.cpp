// Direction dispatch of one level (host code).
#include "dwt2_internal.h"

namespace dwt2 {

hipError_t launch_fwd(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s);
hipError_t launch_inv(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s);
hipError_t launch_adj(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s);

hipError_t launch_level(Direction dir, Wavelet wav, Dtype dt, Scheme sch, int cfg,
                        const LevelParams& p, int planes, hipStream_t stream) {
    if (p.tiles_x <= 0 || p.tiles_y <= 0 || planes <= 0) return hipSuccess;
    if (planes > kMaxGridPlanes || cfg < 0 || cfg >= kNumConfigs) return hipErrorInvalidValue;
    if (kConfigs[cfg].algo == kAlgoLds) return launch_lds(dir, wav, dt, sch, cfg, p, planes, stream);
    if (wav == kDd137 || sch == kSchemePolyconv) return hipErrorInvalidValue;
    if ((sch == kSchemeSeparable || sch == kSchemeFactored) && kConfigs[cfg].algo != kAlgoTile)
        return hipErrorInvalidValue;
    switch (dir) {
        case kForward: return launch_fwd(wav, dt, sch, cfg, p, planes, stream);
        case kInverse: return launch_inv(wav, dt, sch, cfg, p, planes, stream);
        case kAdjoint: return launch_adj(wav, dt, sch, cfg, p, planes, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace dwt2
