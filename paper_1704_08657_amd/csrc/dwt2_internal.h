// Internal interface between the C ABI layer (dwt2_api.cpp) and the HIP
// kernels (dwt2_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dwt2 {

enum Direction : int { kForward = 0, kInverse = 1, kAdjoint = 2 };
enum Wavelet : int { kCdf97 = 0, kCdf53 = 1 };
enum Dtype : int { kF32 = 0, kBF16 = 1, kF16 = 2, kI32 = 3 };

// Tile geometry shared by host planning and the kernels.  A work-group of
// `waves` wave64s owns a tile of kTileBX x (waves * rows) blocks of 2x2
// pixels, of which a halo of kHalo blocks on every side is recomputed and
// discarded.  Each lane holds two horizontally adjacent blocks for `rows`
// consecutive block rows.
constexpr int kLanes = 64;
constexpr int kHalo = 2;
constexpr int kTileBX = 2 * kLanes;                       // 128 blocks
constexpr int kCoreBX = kTileBX - 2 * kHalo;              // 124 blocks

struct TileShape {
    int waves;   // wave64s per work-group, stacked vertically
    int rows;    // block rows per lane
};
constexpr TileShape kTileShapes[] = {{8, 8}, {4, 8}, {8, 4}, {16, 4}, {16, 2}, {4, 4}};
constexpr int kNumTileShapes = 6;
constexpr int kDefaultTileShape = 0;
constexpr int core_rows(TileShape s) { return s.waves * s.rows - 2 * kHalo; }

// One level of a transform.  Forward: `in` is the h x w image of this level,
// `out` the origin of this level's region of the Mallat pyramid (details are
// written there), `out_ll` receives the LL band.  Inverse / adjoint: `in` is
// the pyramid region (details), `in_ll` the LL band, `out` the h x w image.
struct LevelParams {
    const void* in;
    int64_t in_pitch;
    const void* in_ll;
    int64_t in_ll_pitch;
    void* out;
    int64_t out_pitch;
    void* out_ll;
    int64_t out_ll_pitch;
    int32_t h, w;
    int32_t tiles_x, tiles_y;
    int32_t vec;     // 1: every row base is aligned for vector access
};

// Enqueue one level.  Returns hipSuccess or the launch error.
// `shape` indexes kTileShapes; tiles_x / tiles_y of `p` must follow it.
hipError_t launch_level(Direction dir, Wavelet wav, Dtype dt, bool split, int shape,
                        const LevelParams& p, hipStream_t stream);

}  // namespace dwt2
