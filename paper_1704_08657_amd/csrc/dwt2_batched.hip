// Batched forward transform: many images of uneven sizes (dwt2_fwd_batched),
// or a stack of equal planes (dwt2_fwd / dwt2_fwd_planes with
// DWT2_FLAG_PERSISTENT), every level.
//
// One launch per level (the default of dwt2_fwd_batched): a planner kernel
// lays out, from the device copy of the image descriptors, per level an
// exclusive scan of the images' tile counts and every image's LL ping-pong
// buffers; then one launch per level runs every image's tiles of that level.
// Levels are ordered by the kernel boundaries of the stream alone.
//
// One persistent launch (DWT2_FLAG_PERSISTENT): a planner kernel (one work-group) builds the work tables of
// dwt2_batch_plan.h from the image shapes and clears every counter; then one
// persistent launch runs every tile of every level.  Each work-group loops:
// it takes a ticket (one tile) from the sub-queue of the lowest level that
// still has tickets, its own XCD's sub-queue first, then the others; a level
// is entered only once every sub-queue of the level before it is empty, so
// every tile a ticket depends on was handed out before it, to a work-group
// that is already running.  Before a tile of level l >= 1 runs, thread 0
// waits until the chunks of level l - 1 that the tile reads (its rows with
// their halo) report all their tiles finished; the tile then runs the tile
// kernel's body, and its completion is published on its chunk's counter.
// Levels therefore overlap: the first tiles of level l + 1 start while the
// last ones of level l are still running.
//
// Ordering across work-groups, possibly on different XCDs (agent scope):
//   publish: the only data a later tile reads is the LL band of a level
//            below the last, and a tile stores it with agent-scope stores,
//            which the L2 writes through to the point of coherence for the
//            whole device; every wave waits until its stores have
//            completed, the work-group synchronises, thread 0 increments
//            the chunk counter (atomic, agent).  A release fence instead
//            would write back the XCD's whole L2 for every tile;
//   wait:    thread 0 polls the counters (atomic loads, agent scope), the
//            work-group synchronises, every thread fences (acquire, agent:
//            stale cached lines are invalidated) before it loads.
// Every wait is bounded in wall-clock time (wall_limit ticks of the
// constant-rate clock): a wait that runs out raises the error word and the
// abort word of the workspace header, and every later wait returns at once,
// so the launch always ends soon even if a count never arrived; the
// outputs of such a call are invalid and the error word says so.
// Each level keeps its own LL band in the workspace (no ping-pong): a tile
// of level l + 2 may run while a tile of level l + 1 still reads level l's
// band.
#include "dwt2_launch.inl"

#include <stdlib.h>

#include <mutex>

#include "dwt2.h"
#include "dwt2_batch_plan.h"

namespace dwt2 {
namespace kern {
namespace {

constexpr int kPlanThreads = 1024;
constexpr uint32_t kNoTicket = 0xffffffffu;

// Image i of a batch (device array of descriptors) or plane i of a stack.
__device__ __forceinline__ dwt2_image image_at(const ImageSet& S, int i, size_t es) {
    if (S.imgs) return S.imgs[i];
    dwt2_image im;
    im.src = static_cast<const char*>(S.src) + (size_t)i * (size_t)S.src_ps * es;
    im.dst = static_cast<char*>(S.dst) + (size_t)i * (size_t)S.dst_ps * es;
    im.height = S.h;
    im.width = S.w;
    im.src_pitch = S.src_pitch;
    im.dst_pitch = S.dst_pitch;
    return im;
}
__device__ __forceinline__ void image_hw(const ImageSet& S, int i, int32_t* h, int32_t* w) {
    if (S.imgs) {
        *h = S.imgs[i].height;
        *w = S.imgs[i].width;
    } else {
        *h = S.h;
        *w = S.w;
    }
}

// Exclusive scans over the work-group (kPlanThreads threads, 16 wave64s) of
// N values per thread at once: each wave scans with lane shuffles, the wave
// totals meet in LDS; two barriers per call.  tot[k] receives the sum of
// the k-th values over the work-group.
// The last index i in [0, count) with a[i] <= t, for a non-decreasing a
// with a[0] <= t (count and t uniform over the wave).  Every wave searches
// on its own: a pass loads 64 evenly spaced entries of the current segment
// (one per lane, one memory round trip) and keeps the segment after the
// last sample <= t, so up to 64 entries take one pass and up to 4096 two,
// where a binary search takes log2(count) dependent loads.
__device__ __forceinline__ int last_at_most(const uint32_t* a, int count, uint32_t t) {
    const int lane = threadIdx.x & (kLanes - 1);
    int lo = 0, n = count;
    while (n > 1) {
        const int stride = (n + kLanes - 1) / kLanes;
        const int k = lane * stride;
        const bool ok = k < n && a[lo + k] <= t;
        const unsigned long long m = __ballot(ok);     // a prefix of the lanes, lane 0 included
        const int last = 63 - __builtin_clzll(m);
        lo += last * stride;
        n = min(stride, n - last * stride);
    }
    return lo;
}

template <int N, typename U>
__device__ void block_scan(U (&v)[N], U (&tot)[N], U (*wsum)[kPlanThreads / kLanes]) {
    constexpr int kWaves = kPlanThreads / kLanes;
    const int lane = threadIdx.x & (kLanes - 1), w = threadIdx.x / kLanes;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        U x = v[k];
#pragma unroll
        for (int off = 1; off < kLanes; off <<= 1) {
            const U t = __shfl_up(x, off, kLanes);
            if (lane >= off) x += t;
        }
        if (lane == kLanes - 1) wsum[k][w] = x;
        v[k] = x - v[k];                               // exclusive within the wave
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        U before = 0, all = 0;
        for (int j = 0; j < kWaves; ++j) {
            const U s = wsum[k][j];
            before += j < w ? s : U(0);
            all += s;
        }
        v[k] += before;
        tot[k] = all;
    }
    __syncthreads();                                   // wsum is reused by the next call
}

__global__ void __launch_bounds__(kPlanThreads)
persist_plan_kernel(ImageSet S, int count, int levels, int core_cols, int core_rows, int es, BatchLayout BL,
                    unsigned char* ws) {
    __shared__ uint32_t sh32[kXcds][kPlanThreads / kLanes];
    __shared__ uint64_t sh64[1][kPlanThreads / kLanes];
    const int tid = threadIdx.x;
    uint32_t* hdr = reinterpret_cast<uint32_t*>(ws);
    uint32_t* taken = reinterpret_cast<uint32_t*>(ws + BL.off_taken);
    uint32_t* coff = reinterpret_cast<uint32_t*>(ws + BL.off_coff);
    uint32_t* qoff = reinterpret_cast<uint32_t*>(ws + BL.off_qoff);
    uint32_t* cbase = reinterpret_cast<uint32_t*>(ws + BL.off_cbase);
    uint64_t* ll_off = reinterpret_cast<uint64_t*>(ws + BL.off_ll_off);
    uint32_t* done = reinterpret_cast<uint32_t*>(ws + BL.off_done);
    if (tid < 2) hdr[tid] = 0;
    for (int j = tid; j < levels * kXcds; j += kPlanThreads) taken[(size_t)j * kCounterStride] = 0;
    uint32_t base = 0;                             // done counters of the levels so far
    for (int l = 0; l < levels; ++l) {
        uint32_t* crow = coff + (size_t)l * (count + 1);
        uint32_t ccarry = 0, qcarry[kXcds] = {};
        for (int b = 0; b < count; b += kPlanThreads) {
            const int i = b + tid;
            int32_t tx = 0, ty = 0;
            uint32_t c[1] = {0u}, ct[1];
            if (i < count) {
                int32_t h, w, hl, wl;
                image_hw(S, i, &h, &w);
                level_size(h, w, l, &hl, &wl);
                level_tiles(hl, wl, core_cols, core_rows, &tx, &ty);
                c[0] = (uint32_t)chunk_count(ty);
            }
            // the image's first chunk of the level, then its first ticket in every sub-queue
            block_scan<1>(c, ct, sh32);
            const uint32_t g0 = ccarry + c[0];
            uint32_t q[kXcds], qt[kXcds];
#pragma unroll
            for (int y = 0; y < kXcds; ++y) q[y] = i < count ? subqueue_tiles(g0, y, tx, ty) : 0u;
            block_scan<kXcds>(q, qt, sh32);
            if (i < count) {
                crow[i] = g0;
#pragma unroll
                for (int y = 0; y < kXcds; ++y) qoff[((size_t)l * kXcds + y) * (count + 1) + i] = qcarry[y] + q[y];
            }
            ccarry += ct[0];
#pragma unroll
            for (int y = 0; y < kXcds; ++y) qcarry[y] += qt[y];
        }
        if (tid == 0) {
            crow[count] = ccarry;
            cbase[l] = base;
#pragma unroll
            for (int y = 0; y < kXcds; ++y) qoff[((size_t)l * kXcds + y) * (count + 1) + count] = qcarry[y];
        }
        base += ccarry;
    }
    if (tid == 0) cbase[levels] = base;
    // LL bands of every image
    uint64_t carry64 = 0;
    for (int b = 0; b < count; b += kPlanThreads) {
        const int i = b + tid;
        uint64_t v[1] = {0}, t[1];
        if (i < count) {
            int32_t h, w;
            image_hw(S, i, &h, &w);
            v[0] = (uint64_t)image_ll_bytes(h, w, levels, (size_t)es);
        }
        block_scan<1>(v, t, sh64);
        if (i < count) ll_off[i] = carry64 + v[0];
        carry64 += t[0];
    }
    for (uint32_t j = tid; j < base; j += kPlanThreads) done[j] = 0;
}

__device__ __forceinline__ bool is_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---- one launch per level --------------------------------------------------
// Planner: per level an exclusive scan of the images' tile counts (one launch
// of that level covers the tiles of all images) and each image's two LL
// ping-pong buffers.
__global__ void __launch_bounds__(kPlanThreads)
level_plan_kernel(const dwt2_image* imgs, int count, int levels, int core_cols, int core_rows, int es,
                  unsigned char* ws) {
    __shared__ uint32_t sh32[1][kPlanThreads / kLanes];
    __shared__ uint64_t sh64[1][kPlanThreads / kLanes];
    const int tid = threadIdx.x;
    const LevelBatchLayout L = level_batch_layout(count, levels);
    uint32_t* tile_off = reinterpret_cast<uint32_t*>(ws + L.off_tile);
    uint64_t* ll_off = reinterpret_cast<uint64_t*>(ws + L.off_ll_off);
    for (int l = 0; l < levels; ++l) {
        uint32_t* row = tile_off + (size_t)l * (count + 1);
        uint32_t carry = 0;
        for (int b = 0; b < count; b += kPlanThreads) {
            const int i = b + tid;
            uint32_t v[1] = {i < count ? (uint32_t)level_tile_count(imgs[i].height, imgs[i].width, l, core_cols,
                                                                    core_rows)
                                       : 0u};
            uint32_t t[1];
            block_scan<1>(v, t, sh32);
            if (i < count) row[i] = carry + v[0];
            carry += t[0];
        }
        if (tid == 0) row[count] = carry;
    }
    uint64_t carry64 = 0;
    for (int b = 0; b < count; b += kPlanThreads) {
        const int i = b + tid;
        uint64_t v[1] = {i < count ? (uint64_t)pingpong_ll_bytes(imgs[i].height, imgs[i].width, levels, (size_t)es)
                                   : 0ull};
        uint64_t t[1];
        block_scan<1>(v, t, sh64);
        if (i < count) ll_off[i] = carry64 + v[0];
        carry64 += t[0];
    }
}

// Level l of every image.  The grid is a multiple of 8 chunks of
// kLevelChunk tiles; work-groups are dealt round-robin over the 8 XCDs, so
// each XCD is given runs of kLevelChunk consecutive tiles of the level
// (row-major within an image, images in order) and the halo re-reads of
// neighbouring tiles hit its L2.  Levels are ordered by the kernel
// boundaries of the stream: no work-group waits for another.

template <typename T, int SCH, int NW, int K, int BPL>
__global__ void __launch_bounds__(NW * kLanes)
batched_level_kernel(const dwt2_image* imgs, int count, int levels, int l, unsigned char* ws) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    constexpr size_t es = sizeof(T);
    __shared__ TileLds<V, NW, BPL, K> lds;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const LevelBatchLayout L = level_batch_layout(count, levels);
    const uint32_t* off = reinterpret_cast<const uint32_t*>(ws + L.off_tile) + (size_t)l * (count + 1);
    const uint64_t* ll_off = reinterpret_cast<const uint64_t*>(ws + L.off_ll_off);
    unsigned char* ll_area = ws + L.off_ll;

    // XCD x takes chunks x, x + 8, ... of kLevelChunk consecutive tiles
    const uint32_t j = blockIdx.x >> 3;
    const uint32_t t = ((j / kLevelChunk) * 8 + (blockIdx.x & 7)) * kLevelChunk + j % kLevelChunk;
    if (t >= off[count]) return;                  // uniform over the work-group
    // image of tile t: off[] is strictly increasing (every image has a tile)
    const int i = last_at_most(off, count, t);
    const int tt = (int)(t - off[i]);
    const dwt2_image im = imgs[i];

    LevelParams P{};
    int32_t hl, wl;
    level_size(im.height, im.width, l, &hl, &wl);
    P.h = hl;
    P.w = wl;
    level_tiles(hl, wl, Lay<BPL>::CORE_BX, kCoreBY, &P.tiles_x, &P.tiles_y);
    unsigned char* bufA = ll_area + ll_off[i];
    unsigned char* bufB = bufA + pingpong_b_offset(im.height, im.width, levels, es);
    if (l == 0) {
        P.in = im.src;
        P.in_pitch = im.src_pitch;
    } else {
        P.in = (l - 1) % 2 == 0 ? (const void*)bufA : (const void*)bufB;
        P.in_pitch = ll_pitch(wl);
    }
    P.out = im.dst;
    P.out_pitch = im.dst_pitch;
    if (l + 1 == levels) {
        P.out_ll = im.dst;
        P.out_ll_pitch = im.dst_pitch;
    } else {
        P.out_ll = l % 2 == 0 ? (void*)bufA : (void*)bufB;
        P.out_ll_pitch = ll_pitch((wl + 1) / 2);
    }
    P.vec = is_aligned(P.in, 4 * es) && P.in_pitch % 4 == 0 && is_aligned(P.out, BPL * es) &&
            P.out_pitch % BPL == 0 && ((wl + 1) / 2) % BPL == 0 && is_aligned(P.out_ll, BPL * es) &&
            P.out_ll_pitch % BPL == 0;
    P.vec8 = is_aligned(P.in, 2 * es) && P.in_pitch % 2 == 0 && is_aligned(P.out, 2 * es) &&
             P.out_pitch % 2 == 0 && is_aligned(P.out_ll, 2 * es) && P.out_ll_pitch % 2 == 0;
    P.vec16 = is_aligned(P.in, 16) && P.in_pitch % (int64_t)(16 / es) == 0;
    const int ty = tt / P.tiles_x;
    const int tx = tt - ty * P.tiles_x;
    // images whose rows are only 8-byte aligned: semi-vector interior tiles
    // (fused and split steps, as the level kernel)
    if constexpr (SCH == kSchemeFused || SCH == kSchemeSplit) {
        if (!P.vec && P.vec8) {
            tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, true>(P, tx, ty, lds, lane, wv);
            return;
        }
    }
    tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, false>(P, tx, ty, lds, lane, wv);
}

// ---- one persistent launch -------------------------------------------------

// Thread 0: wait until chunks c0..c1 (counters d[], level with tx x ty tiles)
// report all their tiles finished, or give up (see the file comment).
__device__ __attribute__((noinline)) void wait_chunks(const uint32_t* d, int32_t c0, int32_t c1, int32_t tx,
                                                      int32_t ty, uint32_t* hdr, uint64_t wall_limit) {
    const uint64_t t0 = (uint64_t)wall_clock64();
    for (int32_t c = c1; c >= c0; --c) {          // the last chunk is the likeliest to be unfinished
        const uint32_t need = chunk_tiles(c, tx, ty);
        while (__hip_atomic_load(d + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__hip_atomic_load(hdr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
            if ((uint64_t)wall_clock64() - t0 > wall_limit) {
                __hip_atomic_fetch_or(hdr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or(hdr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
}

template <typename T, int SCH, int NW, int K, int BPL>
__global__ void __launch_bounds__(NW * kLanes)
persist_fwd_kernel(ImageSet S, int count, int levels, BatchLayout BL, uint64_t wall_limit, unsigned char* ws) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    constexpr int kCoreBX = Lay<BPL>::CORE_BX;
    constexpr size_t es = sizeof(T);
    static_assert(kCoreBY >= kHalo, "a tile's halo reaches at most one tile row beyond its own");
    __shared__ TileLds<V, NW, BPL, K> lds;
    __shared__ uint32_t sh_ticket[3];
    const int lane = threadIdx.x & (kLanes - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    uint32_t* hdr = reinterpret_cast<uint32_t*>(ws);
    uint32_t* taken = reinterpret_cast<uint32_t*>(ws + BL.off_taken);
    const uint32_t* coff = reinterpret_cast<const uint32_t*>(ws + BL.off_coff);
    const uint32_t* qoff = reinterpret_cast<const uint32_t*>(ws + BL.off_qoff);
    const uint32_t* cbase = reinterpret_cast<const uint32_t*>(ws + BL.off_cbase);
    const uint64_t* ll_off = reinterpret_cast<const uint64_t*>(ws + BL.off_ll_off);
    uint32_t* done = reinterpret_cast<uint32_t*>(ws + BL.off_done);
    unsigned char* ll_area = ws + BL.off_ll;
    const int home = (int)(blockIdx.x & (kXcds - 1));
    int lvl = 0;              // thread 0: lowest level that may still have tickets
    uint32_t empty = 0;       // thread 0: sub-queues of that level found empty

    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t tl = kNoTicket, ty = 0, tp = 0;
            while (lvl < levels && tl == kNoTicket) {
                for (int k = 0; k < kXcds; ++k) {
                    const int y = (home + k) & (kXcds - 1);
                    if (empty & (1u << y)) continue;
                    const uint32_t n = qoff[((size_t)lvl * kXcds + y) * (count + 1) + count];
                    const uint32_t p = n ? __hip_atomic_fetch_add(taken + (size_t)(lvl * kXcds + y) * kCounterStride, 1u,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                         : 0u;
                    if (p < n) {
                        tl = (uint32_t)lvl;
                        ty = (uint32_t)y;
                        tp = p;
                        break;
                    }
                    empty |= 1u << y;
                }
                if (tl == kNoTicket) {
                    ++lvl;
                    empty = 0;
                }
            }
            sh_ticket[0] = tl;
            sh_ticket[1] = ty;
            sh_ticket[2] = tp;
        }
        __syncthreads();
        const uint32_t tl = sh_ticket[0];
        if (tl == kNoTicket) break;                // uniform: every queue is empty
        const int l = (int)tl, y = (int)sh_ticket[1];
        const uint32_t p = sh_ticket[2];
        // the image of ticket p: the last image whose first ticket is <= p
        const uint32_t* q = qoff + ((size_t)l * kXcds + y) * (count + 1);
        const int i = last_at_most(q, count, p);
        const dwt2_image im = image_at(S, i, es);
        int32_t hl, wl, ntx, nty;
        level_size(im.height, im.width, l, &hl, &wl);
        level_tiles(hl, wl, kCoreBX, kCoreBY, &ntx, &nty);
        const uint32_t g0 = coff[(size_t)l * (count + 1) + i];
        int32_t trow, tcol, chunk;
        subqueue_tile(g0, y, ntx, p - q[i], &trow, &tcol, &chunk);
        unsigned char* bands = ll_area + ll_off[i];

        if (l > 0) {
            if (threadIdx.x == 0) {
                int32_t hp, wp, ptx, pty, c0, c1;
                level_size(im.height, im.width, l - 1, &hp, &wp);
                level_tiles(hp, wp, kCoreBX, kCoreBY, &ptx, &pty);
                dep_chunks(trow, kCoreBY, hl, &c0, &c1);
                wait_chunks(done + cbase[l - 1] + coff[(size_t)(l - 1) * (count + 1) + i], c0, c1, ptx, pty, hdr,
                            wall_limit);
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        LevelParams P{};
        P.h = hl;
        P.w = wl;
        P.tiles_x = ntx;
        P.tiles_y = nty;
        if (l == 0) {
            P.in = im.src;
            P.in_pitch = im.src_pitch;
        } else {
            P.in = bands + ll_band_offset(im.height, im.width, l - 1, es);
            P.in_pitch = ll_pitch(wl);
        }
        P.out = im.dst;
        P.out_pitch = im.dst_pitch;
        if (l + 1 == levels) {
            P.out_ll = im.dst;
            P.out_ll_pitch = im.dst_pitch;
        } else {
            P.out_ll = bands + ll_band_offset(im.height, im.width, l, es);
            P.out_ll_pitch = ll_pitch((wl + 1) / 2);
        }
        P.vec = is_aligned(P.in, 4 * es) && P.in_pitch % 4 == 0 && is_aligned(P.out, BPL * es) &&
                P.out_pitch % BPL == 0 && ((wl + 1) / 2) % BPL == 0 && is_aligned(P.out_ll, BPL * es) &&
                P.out_ll_pitch % BPL == 0;
        P.vec8 = is_aligned(P.in, 2 * es) && P.in_pitch % 2 == 0 && is_aligned(P.out, 2 * es) &&
                 P.out_pitch % 2 == 0 && is_aligned(P.out_ll, 2 * es) && P.out_ll_pitch % 2 == 0;
        P.vec16 = is_aligned(P.in, 16) && P.in_pitch % (int64_t)(16 / es) == 0;
        // images whose rows are only 8-byte aligned: semi-vector interior
        // tiles (fused and split steps, as the level kernel)
        bool semi = false;
        if constexpr (SCH == kSchemeFused || SCH == kSchemeSplit) semi = !P.vec && P.vec8;
        // a level that a later one reads stores its LL band with agent-scope
        // stores (written through the L2, see coherent_store)
        const bool read_later = l + 1 < levels;
        if (semi) {
            if (read_later) tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, true, false, true>(P, tcol, trow, lds, lane, wv);
            else tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, true>(P, tcol, trow, lds, lane, wv);
        } else {
            if (read_later) tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, false, false, true>(P, tcol, trow, lds, lane, wv);
            else tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, false>(P, tcol, trow, lds, lane, wv);
        }

        // publish the tile: every wave waits until its stores have completed
        // (the LL band's agent-scope stores are then where every XCD reads
        // them), then thread 0 adds the tile to the chunk counter.  No L2
        // writeback: the band never sits dirty in this XCD's L2.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done + cbase[l] + g0 + chunk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Per device: work-groups of one persistent kernel that fit on the GPU at
// once, and the wall-clock ticks of the wait limit.
struct DeviceInfo {
    int cus = 0;
    uint64_t ticks_per_ms = 0;
};
std::mutex g_info_mu;
DeviceInfo g_info[64];

hipError_t device_info(DeviceInfo* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_info_mu);
    DeviceInfo& d = g_info[dev];
    if (d.cus == 0) {
        int cus = 0, khz = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess) return e;
        d.ticks_per_ms = khz > 0 ? (uint64_t)khz : 100000u;
        d.cus = cus > 0 ? cus : 1;
    }
    *out = d;
    return hipSuccess;
}

// The wall-clock limit of one dependency wait: kWaitLimitMs, or the
// microseconds given in the environment variable DWT2_WAIT_LIMIT_US (tests
// of the failure path set it to 0, so that a wait gives up at once and the
// call reports it).
uint64_t wait_limit_ticks(const DeviceInfo& di) {
    const char* e = getenv("DWT2_WAIT_LIMIT_US");
    if (e && *e) return (uint64_t)strtoull(e, nullptr, 10) * di.ticks_per_ms / 1000u;
    return (uint64_t)kWaitLimitMs * di.ticks_per_ms;
}

template <typename T, int SCH, int NW, int K, int BPL>
hipError_t launch_persist_shape(const ImageSet& S, int count, int levels, void* ws, const BatchLayout& BL,
                                uint64_t tiles, hipStream_t s) {
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    static int per_cu = 0;                        // occupancy of this instantiation (same on every MI355X)
    DeviceInfo di;
    hipError_t e = device_info(&di);
    if (e != hipSuccess) return e;
    if (per_cu == 0) {
        int n = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_fwd_kernel<T, SCH, NW, K, BPL>, NW * kLanes, 0);
        if (e != hipSuccess) return e;
        per_cu = n > 0 ? n : 1;
    }
    unsigned char* w = static_cast<unsigned char*>(ws);
    hipLaunchKernelGGL(persist_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, S, count, levels, Lay<BPL>::CORE_BX,
                       kCoreBY, (int)sizeof(T), BL, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // as many work-groups as fit at once (a multiple of 8, one share per
    // XCD), no more than there are tiles
    uint64_t grid = (uint64_t)di.cus * (uint64_t)per_cu;
    if (grid > tiles) grid = tiles;
    grid = grid < kXcds ? kXcds : grid / kXcds * kXcds;
    hipLaunchKernelGGL((persist_fwd_kernel<T, SCH, NW, K, BPL>), dim3((unsigned)grid), dim3(NW * kLanes), 0, s, S,
                       count, levels, BL, wait_limit_ticks(di), w);
    return hipGetLastError();
}

template <typename T, int SCH, int NW, int K, int BPL>
hipError_t launch_levels_shape(const dwt2_image* dev_imgs, int count, int levels, void* ws,
                               const uint32_t* tiles_per_level, hipStream_t s) {
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    unsigned char* w = static_cast<unsigned char*>(ws);
    hipLaunchKernelGGL(level_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_imgs, count, levels,
                       Lay<BPL>::CORE_BX, kCoreBY, (int)sizeof(T), w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = 0; l < levels; ++l) {
        const uint32_t chunks = (tiles_per_level[l] + kLevelChunk - 1) / kLevelChunk;
        const uint32_t grid = (chunks + 7u) / 8u * 8u * kLevelChunk;
        hipLaunchKernelGGL((batched_level_kernel<T, SCH, NW, K, BPL>), dim3(grid), dim3(NW * kLanes), 0, s,
                           dev_imgs, count, levels, l, w);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int SCH>
hipError_t launch_levels_cfg(int cfg, const dwt2_image* d, int count, int levels, void* ws, const uint32_t* tpl,
                             hipStream_t s) {
    static_assert(kNumConfigs == 10, "dispatch table below lists every kernel configuration");
#define DWT2_LCFG(i)                                                                                 \
    case i:                                                                                          \
        if constexpr (kConfigs[i].algo == kAlgoTile)                                                 \
            return launch_levels_shape<T, SCH, kConfigs[i].waves, kConfigs[i].rows, kConfigs[i].bpl>( \
                d, count, levels, ws, tpl, s);                                                       \
        else                                                                                         \
            return hipErrorInvalidValue;
    switch (cfg) {
        DWT2_LCFG(0) DWT2_LCFG(1) DWT2_LCFG(2) DWT2_LCFG(3) DWT2_LCFG(4) DWT2_LCFG(5) DWT2_LCFG(6) DWT2_LCFG(7)
        DWT2_LCFG(8) DWT2_LCFG(9)
    }
#undef DWT2_LCFG
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_levels_t(Scheme sch, int cfg, const dwt2_image* d, int count, int levels, void* ws,
                           const uint32_t* tpl, hipStream_t s) {
    switch (sch) {
        case kSchemeFused: return launch_levels_cfg<T, kSchemeFused>(cfg, d, count, levels, ws, tpl, s);
        case kSchemeSplit: return launch_levels_cfg<T, kSchemeSplit>(cfg, d, count, levels, ws, tpl, s);
        case kSchemeFactored: return launch_levels_cfg<T, kSchemeFactored>(cfg, d, count, levels, ws, tpl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int SCH>
hipError_t launch_persist_cfg(int cfg, const ImageSet& S, int count, int levels, void* ws, const BatchLayout& BL,
                              uint64_t tiles, hipStream_t s) {
    static_assert(kNumConfigs == 10, "dispatch table below lists every kernel configuration");
#define DWT2_PCFG(i)                                                                                  \
    case i:                                                                                           \
        if constexpr (kConfigs[i].algo == kAlgoTile)                                                  \
            return launch_persist_shape<T, SCH, kConfigs[i].waves, kConfigs[i].rows, kConfigs[i].bpl>( \
                S, count, levels, ws, BL, tiles, s);                                                  \
        else                                                                                          \
            return hipErrorInvalidValue;
    switch (cfg) {
        DWT2_PCFG(0) DWT2_PCFG(1) DWT2_PCFG(2) DWT2_PCFG(3) DWT2_PCFG(4) DWT2_PCFG(5) DWT2_PCFG(6) DWT2_PCFG(7)
        DWT2_PCFG(8) DWT2_PCFG(9)
    }
#undef DWT2_PCFG
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_persist_t(Scheme sch, int cfg, const ImageSet& S, int count, int levels, void* ws,
                            const BatchLayout& BL, uint64_t tiles, hipStream_t s) {
    switch (sch) {
        case kSchemeFused: return launch_persist_cfg<T, kSchemeFused>(cfg, S, count, levels, ws, BL, tiles, s);
        case kSchemeSplit: return launch_persist_cfg<T, kSchemeSplit>(cfg, S, count, levels, ws, BL, tiles, s);
        case kSchemeFactored:
            return launch_persist_cfg<T, kSchemeFactored>(cfg, S, count, levels, ws, BL, tiles, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace kern

bool persist_config_supported(int cfg) { return cfg >= 0 && cfg < kNumConfigs && kConfigs[cfg].algo == kAlgoTile; }

hipError_t launch_fwd_batched_levels(Dtype dt, Scheme sch, int cfg, const dwt2_image* dev_imgs, int count,
                                     int levels, void* ws, const uint32_t* tiles_per_level, hipStream_t s) {
    switch (dt) {
        case kF32: return kern::launch_levels_t<float>(sch, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        case kBF16:
            return kern::launch_levels_t<__hip_bfloat16>(sch, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        case kF16: return kern::launch_levels_t<__half>(sch, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fwd_persistent(Dtype dt, Scheme sch, int cfg, const ImageSet& S, int count, int levels, void* ws,
                                 const BatchLayout& BL, uint64_t tiles, hipStream_t s) {
    switch (dt) {
        case kF32: return kern::launch_persist_t<float>(sch, cfg, S, count, levels, ws, BL, tiles, s);
        case kBF16: return kern::launch_persist_t<__hip_bfloat16>(sch, cfg, S, count, levels, ws, BL, tiles, s);
        case kF16: return kern::launch_persist_t<__half>(sch, cfg, S, count, levels, ws, BL, tiles, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dwt2
