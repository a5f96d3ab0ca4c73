// Work plan of a batched call, shared by the host (argument checks, workspace
// size, grid sizes) and the device (planner and level kernels), so both
// sides derive the same layout from the image descriptors.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dwt2_internal.h"

namespace dwt2 {

// Workspace of a batched call, from its start:
//   uint32 tile_off[levels][count + 1]   first tile of image i within the
//                                        launch of level l; [l][count] = tiles
//                                        of that launch
//   uint64 ll_off[count]                 byte offset of image i's LL buffers
//                                        in the LL area
//   LL area                              per image: buffer A (LL of levels
//                                        1, 3, ...), buffer B (levels 2, 4, ...)
struct BatchLayout {
    size_t off_tile, off_ll_off, off_ll;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline BatchLayout batch_layout(int count, int levels) {
    BatchLayout L;
    L.off_tile = 0;
    L.off_ll_off = align_up(sizeof(uint32_t) * (size_t)levels * (size_t)(count + 1), 256);
    L.off_ll = align_up(L.off_ll_off + sizeof(uint64_t) * (size_t)count, 256);
    return L;
}

// Pitch (elements) of an intermediate LL band of width w.
__host__ __device__ inline int64_t ll_pitch(int32_t w) { return ((int64_t)w + 63) / 64 * 64; }

// Size transformed at level l (0-based) of an h x w image.
__host__ __device__ inline void level_size(int32_t h, int32_t w, int l, int32_t* hl, int32_t* wl) {
    for (int k = 0; k < l; ++k) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
    }
    *hl = h;
    *wl = w;
}

// Tile grid of one level for the tile kernel with `core_cols` x `core_rows`
// output blocks per tile.
__host__ __device__ inline void level_tiles(int32_t hl, int32_t wl, int core_cols, int core_rows, int32_t* tx,
                                            int32_t* ty) {
    const int32_t nEr = (hl + 1) / 2, nEc = (wl + 1) / 2;
    *tx = (nEc + core_cols - 1) / core_cols;
    *ty = (nEr + core_rows - 1) / core_rows;
}

__host__ __device__ inline uint64_t level_tile_count(int32_t h, int32_t w, int l, int core_cols, int core_rows) {
    int32_t hl, wl, tx, ty;
    level_size(h, w, l, &hl, &wl);
    level_tiles(hl, wl, core_cols, core_rows, &tx, &ty);
    return (uint64_t)tx * (uint64_t)ty;
}

// LL band bytes of level l (0-based) of an h x w image.
__host__ __device__ inline size_t ll_band_bytes(int32_t h, int32_t w, int l, size_t es) {
    int32_t hl, wl;
    level_size(h, w, l, &hl, &wl);
    return (size_t)((hl + 1) / 2) * (size_t)ll_pitch((wl + 1) / 2) * es;
}

// Offset of buffer B within an image's LL buffers (a multiple of 256).
__host__ __device__ inline size_t image_ll_b_offset(int32_t h, int32_t w, int levels, size_t es) {
    size_t a = 0;
    for (int l = 0; l + 1 < levels; l += 2) {
        const size_t sz = ll_band_bytes(h, w, l, es);
        a = a > sz ? a : sz;
    }
    return align_up(a, 256);
}

// Bytes of image i's two LL buffers (0 for one level), a multiple of 256.
__host__ __device__ inline size_t image_ll_bytes(int32_t h, int32_t w, int levels, size_t es) {
    size_t b = 0;
    for (int l = 1; l + 1 < levels; l += 2) {
        const size_t sz = ll_band_bytes(h, w, l, es);
        b = b > sz ? b : sz;
    }
    return image_ll_b_offset(h, w, levels, es) + align_up(b, 256);
}

}  // namespace dwt2
