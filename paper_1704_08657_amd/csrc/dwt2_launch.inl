// Launch plumbing shared by the per-direction translation units; included.
#pragma once
#include "dwt2_kernels.inl"

namespace dwt2 {
namespace kern {

template <int DIR, int WAV, typename T, int SCH, int NW, int K, int BPL, bool SEMI, bool LLC = false>
hipError_t launch_grid(const LevelParams& p, int planes, hipStream_t s) {
    // the tiles of all planes, rounded up to a multiple of 8 chunks of
    // kRemapRows tile rows (see level_kernel); planes beyond what one grid
    // holds go to further launches
    const int64_t nt = (int64_t)p.tiles_x * p.tiles_y;
    const int64_t chunk = (int64_t)kRemapRows * p.tiles_x;
    const int64_t limit = 0x7fffffff - 8 * chunk;
    if (nt < 1 || nt > limit) return hipErrorInvalidConfiguration;
    const int64_t per = limit / nt;
    for (int64_t p0 = 0; p0 < planes; p0 += per) {
        LevelParams q = p;
        q.planes = (int32_t)(planes - p0 < per ? planes - p0 : per);
        if (p0 > 0) {
            if (q.in) q.in = static_cast<const T*>(q.in) + p0 * q.in_ps;
            if (q.in_ll) q.in_ll = static_cast<const T*>(q.in_ll) + p0 * q.in_ll_ps;
            if (q.out) q.out = static_cast<T*>(q.out) + p0 * q.out_ps;
            if (q.out_ll) q.out_ll = static_cast<T*>(q.out_ll) + p0 * q.out_ll_ps;
        }
        const int64_t grid = (nt * q.planes + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
        hipLaunchKernelGGL((level_kernel<DIR, WAV, T, SCH, NW, K, BPL, SEMI, LLC>), dim3((unsigned)grid),
                           dim3(NW * kLanes), 0, s, q);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// An image whose rows are 8-byte but not vector aligned runs its interior
// tiles on the semi-vector path (fused and split schemes).  A CDF 9/7 level
// whose output the next level of the call reads stores it with ordinary
// stores on the vector path (ll_cached).
template <int DIR, int WAV, typename T, int SCH, int NW, int K, int BPL>
hipError_t launch_shape(const LevelParams& p, int planes, hipStream_t s) {
    if constexpr (SCH == kSchemeFused || SCH == kSchemeSplit) {
        if (!p.vec && p.vec8) return launch_grid<DIR, WAV, T, SCH, NW, K, BPL, true>(p, planes, s);
    }
    if constexpr (WAV == kCdf97) {
        if (p.ll_cached && p.vec) return launch_grid<DIR, WAV, T, SCH, NW, K, BPL, false, true>(p, planes, s);
    }
    return launch_grid<DIR, WAV, T, SCH, NW, K, BPL, false>(p, planes, s);
}

template <int DIR, int WAV, typename T, bool SPLIT, int W, int PF>
hipError_t launch_stream(const LevelParams& p, int planes, hipStream_t s) {
    const int nt = p.tiles_x * p.tiles_y;
    const int grid = ((nt + 7) >> 3) * 8;
    LevelParams q = p;
    q.planes = planes;
    hipLaunchKernelGGL((stream_kernel<DIR, WAV, T, SPLIT, W, PF>), dim3(grid, planes), dim3(W * kLanes), 0, s, q);
    return hipGetLastError();
}

template <int DIR, int WAV, typename T, int SCH>
hipError_t launch(int cfg, const LevelParams& p, int planes, hipStream_t s) {
    static_assert(kNumConfigs == 10, "dispatch table below lists every kernel configuration");
    // the streaming kernels implement the fused steps (with or without the
    // split); the LDS-plane configurations are dispatched by launch_level
#define DWT2_CFG(i)                                                                              \
    case i:                                                                                      \
        if constexpr (kConfigs[i].algo == kAlgoTile)                                             \
            return launch_shape<DIR, WAV, T, SCH, kConfigs[i].waves, kConfigs[i].rows,           \
                                kConfigs[i].bpl>(p, planes, s);                                  \
        else if constexpr (kConfigs[i].algo == kAlgoStream &&                                    \
                           (SCH == kSchemeFused || SCH == kSchemeSplit))                         \
            return launch_stream<DIR, WAV, T, SCH == kSchemeSplit, kConfigs[i].waves,            \
                                 kConfigs[i].rows>(p, planes, s);                                \
        else                                                                                     \
            return hipErrorInvalidValue;
    switch (cfg) {
        DWT2_CFG(0) DWT2_CFG(1) DWT2_CFG(2) DWT2_CFG(3) DWT2_CFG(4) DWT2_CFG(5) DWT2_CFG(6) DWT2_CFG(7)
        DWT2_CFG(8) DWT2_CFG(9)
    }
#undef DWT2_CFG
    return hipErrorInvalidValue;
}

template <int DIR, int WAV, typename T>
hipError_t launch_float(Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    if constexpr (DIR == kAdjoint) {
        if constexpr (WAV == kCdf97)
            return sch == kSchemeFused ? launch<DIR, WAV, T, kSchemeFused>(cfg, p, planes, s) : hipErrorInvalidValue;
        else
            return hipErrorInvalidValue;          // the adjoint is implemented for CDF 9/7
    } else {
        switch (sch) {
            case kSchemeFused: return launch<DIR, WAV, T, kSchemeFused>(cfg, p, planes, s);
            case kSchemeSplit: return launch<DIR, WAV, T, kSchemeSplit>(cfg, p, planes, s);
            case kSchemeSeparable: return launch<DIR, WAV, T, kSchemeSeparable>(cfg, p, planes, s);
            case kSchemeFactored: return launch<DIR, WAV, T, kSchemeFactored>(cfg, p, planes, s);
            default: return hipErrorInvalidValue;
        }
    }
}

template <int DIR, int WAV>
hipError_t launch_float_dtype(Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    switch (dt) {
        case kF32: return launch_float<DIR, WAV, float>(sch, cfg, p, planes, s);
        case kBF16: return launch_float<DIR, WAV, __hip_bfloat16>(sch, cfg, p, planes, s);
        case kF16: return launch_float<DIR, WAV, __half>(sch, cfg, p, planes, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DIR>
hipError_t launch_dir(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes,
                      hipStream_t s) {
    if (wav == kCdf53) {
        if constexpr (DIR == kAdjoint) {
            return hipErrorInvalidValue;
        } else {
            switch (sch) {
                case kSchemeFused: return launch<DIR, kCdf53, int32_t, kSchemeFused>(cfg, p, planes, s);
                case kSchemeSeparable: return launch<DIR, kCdf53, int32_t, kSchemeSeparable>(cfg, p, planes, s);
                case kSchemeFactored: return launch<DIR, kCdf53, int32_t, kSchemeFactored>(cfg, p, planes, s);
                default: return hipErrorInvalidValue;
            }
        }
    }
    if (wav == kCdf53Real) {
        if constexpr (DIR == kAdjoint) return hipErrorInvalidValue;
        else return launch_float_dtype<DIR, kCdf53Real>(dt, sch, cfg, p, planes, s);
    }
    return launch_float_dtype<DIR, kCdf97>(dt, sch, cfg, p, planes, s);
}

}  // namespace kern
}  // namespace dwt2
