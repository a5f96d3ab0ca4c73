// Launch plumbing shared by the per-direction translation units; included.
#pragma once
#include "dwt2_kernels.inl"

namespace dwt2 {
namespace kern {

template <int DIR, int WAV, typename T, bool SPLIT, int NW, int K, int BPL>
hipError_t launch_shape(const LevelParams& p, int planes, hipStream_t s) {
    // a multiple of 8 chunks of kRemapRows tile rows (see level_kernel)
    const int64_t chunk = (int64_t)kRemapRows * p.tiles_x;
    const int64_t chunks = (p.tiles_y + kRemapRows - 1) / kRemapRows;
    const int64_t grid = (chunks + 7) / 8 * 8 * chunk;
    if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((level_kernel<DIR, WAV, T, SPLIT, NW, K, BPL>), dim3((unsigned)grid, (unsigned)planes),
                       dim3(NW * kLanes), 0, s, p);
    return hipGetLastError();
}

template <int DIR, int WAV, typename T, bool SPLIT, int W, int PF>
hipError_t launch_stream(const LevelParams& p, int planes, hipStream_t s) {
    const int nt = p.tiles_x * p.tiles_y;
    const int grid = ((nt + 7) >> 3) * 8;
    hipLaunchKernelGGL((stream_kernel<DIR, WAV, T, SPLIT, W, PF>), dim3(grid, planes), dim3(W * kLanes), 0, s, p);
    return hipGetLastError();
}

template <int DIR, int WAV, typename T, bool SPLIT>
hipError_t launch(int cfg, const LevelParams& p, int planes, hipStream_t s) {
    static_assert(kNumConfigs == 8, "dispatch table below lists every kernel configuration");
#define DWT2_CFG(i)                                                                              \
    case i:                                                                                      \
        if constexpr (kConfigs[i].algo == kAlgoTile)                                             \
            return launch_shape<DIR, WAV, T, SPLIT, kConfigs[i].waves, kConfigs[i].rows,         \
                                kConfigs[i].bpl>(p, planes, s);                                  \
        else                                                                                     \
            return launch_stream<DIR, WAV, T, SPLIT, kConfigs[i].waves, kConfigs[i].rows>(p, planes, s);
    switch (cfg) {
        DWT2_CFG(0) DWT2_CFG(1) DWT2_CFG(2) DWT2_CFG(3) DWT2_CFG(4) DWT2_CFG(5) DWT2_CFG(6) DWT2_CFG(7)
    }
#undef DWT2_CFG
    return hipErrorInvalidValue;
}

template <int DIR, typename T>
hipError_t launch_float(bool split, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    if constexpr (DIR == kAdjoint) {
        return launch<DIR, kCdf97, T, false>(cfg, p, planes, s);
    } else {
        return split ? launch<DIR, kCdf97, T, true>(cfg, p, planes, s)
                     : launch<DIR, kCdf97, T, false>(cfg, p, planes, s);
    }
}

template <int DIR>
hipError_t launch_dir(Wavelet wav, Dtype dt, bool split, int cfg, const LevelParams& p, int planes,
                      hipStream_t s) {
    if (wav == kCdf53) {
        if constexpr (DIR == kAdjoint) return hipErrorInvalidValue;
        else return launch<DIR, kCdf53, int32_t, false>(cfg, p, planes, s);
    }
    switch (dt) {
        case kF32: return launch_float<DIR, float>(split, cfg, p, planes, s);
        case kBF16: return launch_float<DIR, __hip_bfloat16>(split, cfg, p, planes, s);
        case kF16: return launch_float<DIR, __half>(split, cfg, p, planes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace kern
}  // namespace dwt2
