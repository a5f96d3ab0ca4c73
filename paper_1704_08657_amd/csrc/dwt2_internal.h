// Internal interface between the C ABI layer (dwt2_api.cpp) and the HIP
// kernels (dwt2_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dwt2.h"

namespace dwt2 {

enum Direction : int { kForward = 0, kInverse = 1, kAdjoint = 2 };
// kCdf53: the reversible integer CDF 5/3; kCdf53Real: the real-valued one
enum Wavelet : int { kCdf97 = 0, kCdf53 = 1, kCdf53Real = 2, kDd137 = 3 };
enum Dtype : int { kF32 = 0, kBF16 = 1, kF16 = 2, kI32 = 3 };
// Lifting scheme of a level: the fused non-separable steps, the fused steps
// with the P0/P1 split, the separable steps (the comparison scheme: every
// fused step replaced by its horizontal and its vertical step, a barrier
// each), or the fused steps evaluated as those two factors in registers (one
// barrier per fused step: the horizontal factor never leaves the wave).
// The LDS-plane kernel (kAlgoLds) also runs the non-separable
// polyconvolution: one step N_{P,U} per lifting pair.
enum Scheme : int { kSchemeFused = 0, kSchemeSplit = 1, kSchemeSeparable = 2, kSchemeFactored = 3,
                    kSchemePolyconv = 4 };

// Geometry shared by host planning and the kernels, in blocks of 2x2 pixels.
// A tile (kAlgoTile) has 64 * bpl output columns (bpl blocks per lane) and
// waves * rows - 2 * kHalo output rows; a halo of kHalo blocks on every side
// is recomputed and discarded.  A stream strip (kAlgoStream) has 124 output
// columns.
constexpr int kLanes = 64;
constexpr int kHalo = 2;
constexpr int kStreamCoreBX = 2 * kLanes - 2 * kHalo;     // stream kernel: 124 (halo in the edge lanes)

// Kernel configurations.
//  kAlgoTile:   one work-group = `waves` wave64s stacked vertically, one tile
//               of (64 * bpl) x (waves * rows) blocks held in VGPRs (`rows`
//               block rows and `bpl` block columns per lane, plus a halo
//               pair), one barrier per fused step.
//  kAlgoStream: every wave64 walks down its own column strip of 128 blocks,
//               `rows` block rows of loads in flight ahead of the computation;
//               `waves` strips per work-group; `seg` block rows per segment.
//  kAlgoLds:    the tile with its halo held as the four polyphase planes
//               in LDS (double-buffered), every step a 2-D stencil over them
//               with one barrier; `cx` x `cy` output blocks per work-group of
//               `waves` wave64s.  Runs any step program: fused, separable
//               and polyconvolution schemes, two-tap and four-tap filters.
enum Algo : int { kAlgoTile = 0, kAlgoStream = 1, kAlgoLds = 2 };
struct KernelConfig {
    int algo;
    int waves;
    int rows;
    int seg;
    int bpl;    // kAlgoTile: block columns per lane (2 or 4)
    int cx, cy; // kAlgoLds: output blocks of one work-group tile
};
constexpr KernelConfig kConfigs[] = {
    {kAlgoTile, 4, 4, 0, 2, 0, 0},    {kAlgoTile, 8, 4, 0, 2, 0, 0},    {kAlgoTile, 4, 4, 0, 4, 0, 0},
    {kAlgoTile, 4, 6, 0, 2, 0, 0},    {kAlgoTile, 8, 2, 0, 4, 0, 0},    {kAlgoStream, 4, 8, 64, 2, 0, 0},
    {kAlgoStream, 1, 8, 64, 2, 0, 0}, {kAlgoStream, 4, 8, 32, 2, 0, 0}, {kAlgoLds, 4, 0, 0, 0, 64, 16},
    {kAlgoLds, 4, 0, 0, 0, 32, 32}};
constexpr int kNumConfigs = 10;
constexpr int kDefaultConfig = 0;
constexpr int kDefaultLdsConfig = 8;
// Tile kernels deal work over the 8 XCDs in chunks of kRemapRows tile rows;
// the grid is a multiple of 8 chunks.
constexpr int kRemapRows = 2;
// output block rows / columns of one tile (kAlgoTile, kAlgoLds)
constexpr int core_rows(KernelConfig c) { return c.algo == kAlgoLds ? c.cy : c.waves * c.rows - 2 * kHalo; }
constexpr int core_cols(KernelConfig c) { return c.algo == kAlgoLds ? c.cx : kLanes * c.bpl; }
// samples per vector access of a subband row (alignment the `vec` path needs)
constexpr int subband_vec(KernelConfig c) { return c.algo == kAlgoTile ? c.bpl : 2; }

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
    int32_t vec;       // 1: every row base is aligned for vector access
    int32_t seg_rows;  // kAlgoStream: block rows per segment
    // Plane batch: the launch covers `planes` planes; plane p's buffers
    // start p * (stride) elements after those of plane 0.  Set by the
    // launcher (the tile kernel deals the tiles of all planes as one list,
    // the streaming kernel takes one grid row per plane).
    int64_t in_ps, in_ll_ps, out_ps, out_ll_ps;
    int32_t planes;
    // Without `vec`: every row base (and plane stride) is 8-byte aligned
    // (even pitches), so interior tiles can use pairs of samples (the
    // semi-vector interior path).
    int32_t vec8;
    // With `vec`: the image rows (forward input, inverse / adjoint output)
    // start 16-byte aligned, so 16-bit samples of 4 blocks per lane move as
    // one 16-byte access per row.
    int32_t vec16;
    // CDF 9/7, a level whose output the call's next level reads (forward:
    // the LL band of every level but the last; inverse / adjoint: the image
    // of every level but the finest): interior tiles store it with ordinary
    // stores, so the next level finds it in the caches; every other store
    // stays nontemporal.  Read by the launcher, which picks the kernel
    // variant.
    int32_t ll_cached;
};

// Enqueue one level for `planes` planes (1 <= planes <= kMaxGridPlanes).
// Returns hipSuccess or the launch error.  `cfg` indexes kConfigs;
// tiles_x / tiles_y (and seg_rows) of `p` must follow it: for kAlgoTile the
// tile grid, for kAlgoStream the number of strip groups (ceil(strips /
// waves)) and of segments.
constexpr int kMaxGridPlanes = 65535;
// kSchemeSeparable and kSchemeFactored run on the tile configurations only.
hipError_t launch_level(Direction dir, Wavelet wav, Dtype dt, Scheme scheme, int cfg,
                        const LevelParams& p, int planes, hipStream_t stream);
// The LDS-plane kernel (kConfigs[cfg].algo == kAlgoLds): forward and inverse
// of the float wavelets, fused / separable / polyconvolution schemes.
hipError_t launch_lds(Direction dir, Wavelet wav, Dtype dt, Scheme scheme, int cfg, const LevelParams& p,
                      int planes, hipStream_t stream);

}  // namespace dwt2
