// Work plans of the batched forward transform, shared by the host (argument
// checks, workspace size, grid sizes), the planner and transform kernels,
// and the host checks in tests/host, so all of them derive the same tables
// from the image shapes.  Two plans: one launch per level for all images
// (default), and one persistent launch for every level (a batch of images of
// any sizes, or a stack of equal planes).
//
// Persistent work units.  Level l of image i is cut into the tiles of the tile kernel
// (core_cols x core_rows output blocks).  Pairs of tile rows form a chunk;
// the chunks of a level are numbered image after image, and chunk g goes to
// sub-queue g % 8 (one per XCD: work-group b is expected on XCD b % 8 and
// serves its own sub-queue first, so neighbouring tiles, whose halos overlap,
// meet in one L2).  A ticket is one tile: ticket p of sub-queue (l, y) is
// the p-th tile of that sub-queue's chunks in order.  A chunk is also the
// unit of completion: done[] counts its finished tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dwt2_internal.h"

namespace dwt2 {

constexpr int kXcds = 8;          // sub-queues per level
constexpr int kChunkRows = 2;     // tile rows per chunk
constexpr int kCounterStride = 32;  // uint32 between two ticket counters (one 128-byte line each)

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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

// Chunks of a level with ty tile rows, and the tiles of chunk c.
__host__ __device__ inline int32_t chunk_count(int32_t ty) { return (ty + kChunkRows - 1) / kChunkRows; }
__host__ __device__ inline uint32_t chunk_tiles(int32_t c, int32_t tx, int32_t ty) {
    const int32_t rows = ty - c * kChunkRows < kChunkRows ? ty - c * kChunkRows : kChunkRows;
    return (uint32_t)rows * (uint32_t)tx;
}

// First chunk of an image (level-local number g0) that lands in sub-queue y.
__host__ __device__ inline int32_t first_chunk_in(uint32_t g0, int y) {
    return (int32_t)(((uint32_t)y + kXcds - g0 % kXcds) % kXcds);
}

// Tiles of one image-level (first chunk number g0) in sub-queue y.
__host__ __device__ inline uint32_t subqueue_tiles(uint32_t g0, int y, int32_t tx, int32_t ty) {
    const int32_t n = chunk_count(ty), c0 = first_chunk_in(g0, y);
    if (c0 >= n) return 0;
    const int32_t cnt = (n - c0 + kXcds - 1) / kXcds;          // chunks c0, c0 + 8, ... below n
    uint32_t t = (uint32_t)cnt * kChunkRows * (uint32_t)tx;
    if ((n - 1 - c0) % kXcds == 0) t -= kChunkRows * (uint32_t)tx - chunk_tiles(n - 1, tx, ty);
    return t;
}

// The q-th tile of an image-level in sub-queue y: its tile row and column
// and its chunk.
__host__ __device__ inline void subqueue_tile(uint32_t g0, int y, int32_t tx, uint32_t q, int32_t* row,
                                              int32_t* col, int32_t* chunk) {
    const uint32_t per = kChunkRows * (uint32_t)tx;
    const int32_t c = first_chunk_in(g0, y) + kXcds * (int32_t)(q / per);
    const uint32_t r = q % per;
    *chunk = c;
    *row = c * kChunkRows + (int32_t)(r / (uint32_t)tx);
    *col = (int32_t)(r % (uint32_t)tx);
}

// Whole-point symmetric extension of a row index r into [0, n), n >= 2
// (periodic with period 2 (n - 1)), as the tile kernel's border loads take it.
__host__ __device__ inline int64_t reflect_row(int64_t r, int64_t n) {
    if (r >= 0 && r < n) return r;
    const int64_t period = 2 * (n - 1);
    int64_t q = r % period;
    if (q < 0) q += period;
    return q < n ? q : period - q;
}

// The chunks [*first, *last] of level l-1 whose LL rows a tile of level l
// in tile row `row` loads: its core block rows with a halo of kHalo blocks on
// each side, i.e. input rows [lo, hi), each taken at its reflected position
// (a tile past the image's bottom loads rows from far up the image; they do
// not reach its stored outputs, but they are read, so they are waited for
// too).  LL row r of level l-1 is written by its tile row r / core_rows.
// hl = height of level l.
__host__ __device__ inline void dep_chunks(int32_t row, int core_rows, int32_t hl, int32_t* first, int32_t* last) {
    const int64_t lo = 2 * ((int64_t)row * core_rows - kHalo), hi = 2 * ((int64_t)(row + 1) * core_rows + kHalo);
    int64_t a, b;
    if (lo >= 0 && hi <= hl) {
        a = lo;
        b = hi - 1;
    } else {
        a = hl;
        b = -1;
        for (int64_t r = lo; r < hi; ++r) {
            const int64_t q = reflect_row(r, hl);
            a = q < a ? q : a;
            b = q > b ? q : b;
        }
    }
    *first = (int32_t)(a / ((int64_t)core_rows * kChunkRows));
    *last = (int32_t)(b / ((int64_t)core_rows * kChunkRows));
}

// LL band bytes of level l (0-based) of an h x w image, and the bytes of one
// image's bands: every level but the last keeps its own band (256-byte
// aligned), so no level overwrites what an unfinished tile of the next
// level still reads.
__host__ __device__ inline size_t ll_band_bytes(int32_t h, int32_t w, int l, size_t es) {
    int32_t hl, wl;
    level_size(h, w, l, &hl, &wl);
    return align_up((size_t)((hl + 1) / 2) * (size_t)ll_pitch((wl + 1) / 2) * es, 256);
}
__host__ __device__ inline size_t ll_band_offset(int32_t h, int32_t w, int l, size_t es) {
    size_t o = 0;
    for (int k = 0; k < l; ++k) o += ll_band_bytes(h, w, k, es);
    return o;
}
__host__ __device__ inline size_t image_ll_bytes(int32_t h, int32_t w, int levels, size_t es) {
    return ll_band_offset(h, w, levels - 1, es);
}

// ---- one launch per level (the default path of dwt2_fwd_batched) ----------
// Workspace, from its start:
//   uint32 tile_off[levels][count + 1]   first tile of image i within the
//                                        launch of level l; [l][count] = tiles
//                                        of that launch
//   uint64 ll_off[count]                 byte offset of image i's LL buffers
//                                        in the LL area
//   LL area                              per image: buffer A (LL of levels
//                                        1, 3, ...), buffer B (levels 2, 4, ...)
// The batched level kernel deals its grid over the 8 XCDs in chunks of this
// many consecutive tiles.
constexpr int kLevelChunk = 64;

struct LevelBatchLayout {
    size_t off_tile, off_ll_off, off_ll;
};

__host__ __device__ inline LevelBatchLayout level_batch_layout(int count, int levels) {
    LevelBatchLayout L;
    L.off_tile = 0;
    L.off_ll_off = align_up(sizeof(uint32_t) * (size_t)levels * (size_t)(count + 1), 256);
    L.off_ll = align_up(L.off_ll_off + sizeof(uint64_t) * (size_t)count, 256);
    return L;
}

// Offset of buffer B within an image's ping-pong LL buffers (a multiple of 256).
__host__ __device__ inline size_t pingpong_b_offset(int32_t h, int32_t w, int levels, size_t es) {
    size_t a = 0;
    for (int l = 0; l + 1 < levels; l += 2) {
        const size_t sz = ll_band_bytes(h, w, l, es);
        a = a > sz ? a : sz;
    }
    return a;
}

// Bytes of an image's two ping-pong LL buffers (0 for one level).
__host__ __device__ inline size_t pingpong_ll_bytes(int32_t h, int32_t w, int levels, size_t es) {
    size_t b = 0;
    for (int l = 1; l + 1 < levels; l += 2) {
        const size_t sz = ll_band_bytes(h, w, l, es);
        b = b > sz ? b : sz;
    }
    return pingpong_b_offset(h, w, levels, es) + b;
}

// ---- one persistent launch (DWT2_FLAG_PERSISTENT) --------------------------
// Workspace of a persistent call, from its start:
//   header: uint32 error (a dependency wait ran out of time), uint32 abort
//   uint32 taken[levels][8] (kCounterStride apart)   next ticket of each sub-queue
//   uint32 coff[levels][count + 1]      first chunk of image i at level l
//   uint32 qoff[levels][8][count + 1]   first ticket of image i in sub-queue (l, y)
//   uint32 cbase[levels + 1]            first done counter of level l
//   uint64 ll_off[count]                offset of image i's LL bands in the LL area
//   uint32 done[chunks]                 finished tiles of every chunk
//   LL area
struct BatchLayout {
    size_t off_taken, off_coff, off_qoff, off_cbase, off_ll_off, off_done, off_ll;
};
constexpr size_t kHeaderBytes = 256;

// Layout for `count` images with `chunks` chunks over all levels.
__host__ __device__ inline BatchLayout batch_layout(int count, int levels, uint64_t chunks) {
    BatchLayout L;
    L.off_taken = kHeaderBytes;
    L.off_coff = L.off_taken + sizeof(uint32_t) * kCounterStride * (size_t)levels * kXcds;
    L.off_qoff = L.off_coff + sizeof(uint32_t) * (size_t)levels * (size_t)(count + 1);
    L.off_cbase = L.off_qoff + sizeof(uint32_t) * (size_t)levels * kXcds * (size_t)(count + 1);
    L.off_ll_off = align_up(L.off_cbase + sizeof(uint32_t) * (size_t)(levels + 1), 8);
    L.off_done = L.off_ll_off + sizeof(uint64_t) * (size_t)count;
    L.off_ll = align_up(L.off_done + sizeof(uint32_t) * (size_t)chunks, 256);
    return L;
}

// The images of one persistent call: a batch (a device array of
// descriptors) or a stack of equal planes (plane i at i * plane stride).
struct ImageSet {
    const dwt2_image* imgs;      // batch; nullptr for a plane stack
    const void* src;             // plane stack: plane 0 of the source and destination
    void* dst;
    int64_t src_ps, dst_ps;      // plane strides (elements)
    int64_t src_pitch, dst_pitch;
    int32_t h, w;
};

// A dependency wait that lasts longer than this is taken as a failure (the
// call's error word is raised and its outputs are invalid).
constexpr int kWaitLimitMs = 200;

// Planner plus one launch per level for a tile kernel configuration
// (persist_config_supported), CDF 9/7 forward, fused, split or factored
// steps, float storage; `tiles_per_level[l]` (host array) is the number of tiles of level l
// summed over the images and sizes that level's grid.
hipError_t launch_fwd_batched_levels(Dtype dt, Scheme sch, int cfg, const dwt2_image* dev_imgs, int count,
                                     int levels, void* ws, const uint32_t* tiles_per_level, hipStream_t s);

// Planner plus persistent kernel for a tile kernel configuration
// (persist_config_supported), CDF 9/7 forward with the fused, split or
// factored steps, float storage.  `BL` from batch_layout with the chunks of this
// configuration, `tiles` the tiles of all levels and images.
bool persist_config_supported(int cfg);
hipError_t launch_fwd_persistent(Dtype dt, Scheme sch, int cfg, const ImageSet& S, int count, int levels, void* ws,
                                 const BatchLayout& BL, uint64_t tiles, hipStream_t s);

}  // namespace dwt2
