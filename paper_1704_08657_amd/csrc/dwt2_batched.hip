// Batched forward transform: many images of uneven sizes, every level, in a
// fixed sequence of launches on one stream.
//
// A planner kernel lays out the work from the device copy of the image
// descriptors: for every level an exclusive scan of the images' tile counts
// (so one launch of that level covers the tiles of all images), and each
// image's two LL ping-pong buffers in the workspace.  Then one launch per
// level runs every image's tiles of that level; a work-group finds its image
// by a binary search of the level's scan.  Levels are ordered by the kernel
// boundaries of the stream alone: no work-group ever waits for another, and
// there are no atomics.  The call performs no copies or allocations, so the
// sequence can be captured in a graph and replayed.
#include "dwt2_launch.inl"

#include "dwt2.h"
#include "dwt2_batch_plan.h"

namespace dwt2 {
namespace kern {
namespace {

constexpr int kPlanThreads = 1024;

// Block-wide inclusive scan of one value per thread; *total receives the sum.
template <typename U>
__device__ U block_scan(U v, U* sh, U* total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const U t = tid >= off ? sh[tid - off] : U(0);
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    const U r = sh[tid];
    *total = sh[kPlanThreads - 1];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kPlanThreads)
batch_plan_kernel(const dwt2_image* imgs, int count, int levels, int core_cols, int core_rows, int es,
                  unsigned char* ws) {
    __shared__ uint32_t sh32[kPlanThreads];
    __shared__ uint64_t sh64[kPlanThreads];
    const int tid = threadIdx.x;
    const BatchLayout L = batch_layout(count, levels);
    uint32_t* tile_off = reinterpret_cast<uint32_t*>(ws + L.off_tile);
    uint64_t* ll_off = reinterpret_cast<uint64_t*>(ws + L.off_ll_off);
    for (int l = 0; l < levels; ++l) {
        uint32_t* row = tile_off + (size_t)l * (count + 1);
        uint32_t carry = 0;
        for (int base = 0; base < count; base += kPlanThreads) {
            const int i = base + tid;
            const uint32_t v = i < count ? (uint32_t)level_tile_count(imgs[i].height, imgs[i].width, l, core_cols, core_rows) : 0u;
            uint32_t tot;
            const uint32_t inc = block_scan(v, sh32, &tot);
            if (i < count) row[i] = carry + inc - v;
            carry += tot;
        }
        if (tid == 0) row[count] = carry;
    }
    uint64_t carry64 = 0;
    for (int base = 0; base < count; base += kPlanThreads) {
        const int i = base + tid;
        const uint64_t v = i < count ? (uint64_t)image_ll_bytes(imgs[i].height, imgs[i].width, levels, es) : 0ull;
        uint64_t tot;
        const uint64_t inc = block_scan(v, sh64, &tot);
        if (i < count) ll_off[i] = carry64 + inc - v;
        carry64 += tot;
    }
}

__device__ __forceinline__ bool is_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Level l of every image.  The grid is a multiple of 8 chunks of kBatchChunk
// tiles; work-groups are dealt round-robin over the 8 XCDs, so each XCD is
// given runs of kBatchChunk consecutive tiles of the level (row-major within
// an image, images in order) and the halo re-reads of neighbouring tiles hit
// its L2.
template <typename T, bool SPLIT, int NW, int K, int BPL>
__global__ void __launch_bounds__(NW * kLanes)
batched_level_kernel(const dwt2_image* imgs, int count, int levels, int l, unsigned char* ws) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    constexpr size_t es = sizeof(T);
    __shared__ TileLds<V, NW, BPL, K> lds;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const BatchLayout L = batch_layout(count, levels);
    const uint32_t* off = reinterpret_cast<const uint32_t*>(ws + L.off_tile) + (size_t)l * (count + 1);
    const uint64_t* ll_off = reinterpret_cast<const uint64_t*>(ws + L.off_ll_off);
    unsigned char* ll_area = ws + L.off_ll;

    // XCD x takes chunks x, x + 8, ... of kBatchChunk consecutive tiles
    const uint32_t j = blockIdx.x >> 3;
    const uint32_t t = ((j / kBatchChunk) * 8 + (blockIdx.x & 7)) * kBatchChunk + j % kBatchChunk;
    if (t >= off[count]) return;                  // uniform over the work-group
    // image of tile t: off[] is strictly increasing (every image has a tile)
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid;
    }
    const int i = lo;
    const int tt = (int)(t - off[i]);
    const dwt2_image im = imgs[i];

    LevelParams P{};
    int32_t hl, wl;
    level_size(im.height, im.width, l, &hl, &wl);
    P.h = hl;
    P.w = wl;
    level_tiles(hl, wl, Lay<BPL>::CORE_BX, kCoreBY, &P.tiles_x, &P.tiles_y);
    unsigned char* bufA = ll_area + ll_off[i];
    unsigned char* bufB = bufA + image_ll_b_offset(im.height, im.width, levels, es);
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
    const int ty = tt / P.tiles_x;
    const int tx = tt - ty * P.tiles_x;
    // images whose rows are only 8-byte aligned: semi-vector interior tiles
    constexpr int SCH = SPLIT ? kSchemeSplit : kSchemeFused;
    if (!P.vec && P.vec8) tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, true>(P, tx, ty, lds, lane, wv);
    else tile_body<kForward, kCdf97, T, SCH, NW, K, BPL, false>(P, tx, ty, lds, lane, wv);
}

template <typename T, bool SPLIT, int NW, int K, int BPL>
hipError_t launch_batched_shape(const dwt2_image* dev_imgs, int count, int levels, void* ws,
                                const uint32_t* tiles_per_level, hipStream_t s) {
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    unsigned char* w = static_cast<unsigned char*>(ws);
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_imgs, count, levels,
                       Lay<BPL>::CORE_BX, kCoreBY, (int)sizeof(T), w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = 0; l < levels; ++l) {
        const uint32_t chunks = (tiles_per_level[l] + kBatchChunk - 1) / kBatchChunk;
        const uint32_t grid = (chunks + 7u) / 8u * 8u * kBatchChunk;
        hipLaunchKernelGGL((batched_level_kernel<T, SPLIT, NW, K, BPL>), dim3(grid), dim3(NW * kLanes), 0, s, dev_imgs,
                           count, levels, l, w);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool SPLIT>
hipError_t launch_batched_cfg(int cfg, const dwt2_image* d, int count, int levels, void* ws, const uint32_t* tpl,
                              hipStream_t s) {
    static_assert(kNumConfigs == 10, "dispatch table below lists every kernel configuration");
#define DWT2_BCFG(i)                                                                               \
    case i:                                                                                        \
        if constexpr (kConfigs[i].algo == kAlgoTile)                                               \
            return launch_batched_shape<T, SPLIT, kConfigs[i].waves, kConfigs[i].rows, kConfigs[i].bpl>( \
                d, count, levels, ws, tpl, s);                                                     \
        else                                                                                       \
            return hipErrorInvalidValue;
    switch (cfg) {
        DWT2_BCFG(0) DWT2_BCFG(1) DWT2_BCFG(2) DWT2_BCFG(3) DWT2_BCFG(4) DWT2_BCFG(5) DWT2_BCFG(6) DWT2_BCFG(7)
        DWT2_BCFG(8) DWT2_BCFG(9)
    }
#undef DWT2_BCFG
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batched_t(bool split, int cfg, const dwt2_image* d, int count, int levels, void* ws,
                            const uint32_t* tpl, hipStream_t s) {
    return split ? launch_batched_cfg<T, true>(cfg, d, count, levels, ws, tpl, s)
                 : launch_batched_cfg<T, false>(cfg, d, count, levels, ws, tpl, s);
}

}  // namespace
}  // namespace kern

bool batched_config_supported(int cfg) { return cfg >= 0 && cfg < kNumConfigs && kConfigs[cfg].algo == kAlgoTile; }

hipError_t launch_fwd_batched(Dtype dt, bool split, int cfg, const dwt2_image* dev_imgs, int count, int levels,
                              void* ws, const uint32_t* tiles_per_level, hipStream_t s) {
    switch (dt) {
        case kF32: return kern::launch_batched_t<float>(split, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        case kBF16:
            return kern::launch_batched_t<__hip_bfloat16>(split, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        case kF16: return kern::launch_batched_t<__half>(split, cfg, dev_imgs, count, levels, ws, tiles_per_level, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dwt2
