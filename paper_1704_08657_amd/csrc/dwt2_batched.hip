// Batched forward transform: many images of uneven sizes, every level, in one
// persistent launch.
//
// A planner kernel lays out the work from the device copy of the image
// descriptors: for every (level, image) the number of chunks of
// kChunkTiles tiles, numbered level-major (all images' level 1, then all
// level 2, ...), and each image's two LL ping-pong buffers in the workspace.
// The persistent kernel then loops: a work-group takes the next ticket from
// one counter, finds its (level, image, chunk), waits until every tile of the
// same image's previous level has been published, runs the tiles (the tile
// kernel's body), and publishes them.  A wait only ever refers to smaller
// tickets, which were taken by work-groups that are already running, so the
// queue cannot deadlock; every wait is also bounded, and a wait that runs out
// of patience raises a flag in the workspace header instead of hanging.
// Everything runs on the caller's stream with no host copies, so the pair of
// launches can be captured in a graph and replayed.
#include "dwt2_launch.inl"

#include "dwt2.h"
#include "dwt2_batch_plan.h"

namespace dwt2 {
namespace kern {
namespace {

constexpr int kPlanThreads = 1024;
constexpr uint32_t kWaitSpins = 1u << 22;   // each spin sleeps briefly; bounded in total

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
batch_plan_kernel(const dwt2_image* imgs, int count, int levels, int core_rows, int es, unsigned char* ws) {
    __shared__ uint32_t sh32[kPlanThreads];
    __shared__ uint64_t sh64[kPlanThreads];
    const int tid = threadIdx.x;
    const BatchLayout L = batch_layout(count, levels);
    BatchHeader* hd = reinterpret_cast<BatchHeader*>(ws);
    uint32_t* chunk_off = reinterpret_cast<uint32_t*>(ws + L.off_chunk);
    uint32_t* done = reinterpret_cast<uint32_t*>(ws + L.off_done);
    uint64_t* ll_off = reinterpret_cast<uint64_t*>(ws + L.off_ll_off);
    for (int j = tid; j < levels * count; j += kPlanThreads) done[j] = 0;
    // first ticket of every (level, image), level-major
    uint32_t carry = 0;
    for (int l = 0; l < levels; ++l) {
        for (int base = 0; base < count; base += kPlanThreads) {
            const int i = base + tid;
            const uint32_t v = i < count ? level_chunks(imgs[i].height, imgs[i].width, l, core_rows) : 0u;
            uint32_t tot;
            const uint32_t inc = block_scan(v, sh32, &tot);
            if (i < count) chunk_off[l * count + i] = carry + inc - v;
            carry += tot;
        }
    }
    // LL buffers of every image
    uint64_t carry64 = 0;
    for (int base = 0; base < count; base += kPlanThreads) {
        const int i = base + tid;
        const uint64_t v = i < count ? (uint64_t)image_ll_bytes(imgs[i].height, imgs[i].width, levels, es) : 0ull;
        uint64_t tot;
        const uint64_t inc = block_scan(v, sh64, &tot);
        if (i < count) ll_off[i] = carry64 + inc - v;
        carry64 += tot;
    }
    if (tid == 0) {
        chunk_off[levels * count] = carry;
        hd->next = 0;
        hd->error = 0;
        hd->total = carry;
        hd->count = (uint32_t)count;
        hd->levels = (uint32_t)levels;
    }
}

__device__ __forceinline__ bool is_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

template <typename T, bool SPLIT, int NW, int K>
__global__ void __launch_bounds__(NW * kLanes)
batched_fwd_kernel(const dwt2_image* imgs, int count, int levels, unsigned char* ws) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    constexpr size_t es = sizeof(T);
    __shared__ Edge8<V> bufT[NW][kLanes];
    __shared__ Edge8<V> bufS[NW][kLanes];
    __shared__ uint32_t sh_ticket;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const BatchLayout L = batch_layout(count, levels);
    BatchHeader* hd = reinterpret_cast<BatchHeader*>(ws);
    const uint32_t* chunk_off = reinterpret_cast<const uint32_t*>(ws + L.off_chunk);
    uint32_t* done = reinterpret_cast<uint32_t*>(ws + L.off_done);
    const uint64_t* ll_off = reinterpret_cast<const uint64_t*>(ws + L.off_ll_off);
    unsigned char* ll_area = ws + L.off_ll;
    const int entries = levels * count;
    const uint32_t total = chunk_off[entries];

    for (;;) {
        if (threadIdx.x == 0) sh_ticket = atomicAdd(&hd->next, 1u);
        __syncthreads();
        const uint32_t t = sh_ticket;
        __syncthreads();
        if (t >= total) break;
        // (level, image) of the ticket: chunk_off is strictly increasing
        int lo = 0, hi = entries;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (chunk_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int l = lo / count;
        const int i = lo - l * count;
        const uint32_t chunk = t - chunk_off[lo];
        const dwt2_image im = imgs[i];

        LevelParams P{};
        int32_t hl, wl;
        level_size(im.height, im.width, l, &hl, &wl);
        P.h = hl;
        P.w = wl;
        level_tiles(hl, wl, kCoreBY, &P.tiles_x, &P.tiles_y);
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
        P.vec = is_aligned(P.in, 4 * es) && P.in_pitch % 4 == 0 && is_aligned(P.out, 2 * es) &&
                P.out_pitch % 2 == 0 && ((wl + 1) / 2) % 2 == 0 && is_aligned(P.out_ll, 2 * es) &&
                P.out_ll_pitch % 2 == 0;

        // every tile of this image's previous level must be published
        if (l > 0) {
            if (threadIdx.x == 0) {
                int32_t hp, wp, txp, typ;
                level_size(im.height, im.width, l - 1, &hp, &wp);
                level_tiles(hp, wp, kCoreBY, &txp, &typ);
                const uint32_t need = (uint32_t)txp * (uint32_t)typ;
                uint32_t* flag = &done[(l - 1) * count + i];
                uint32_t spins = 0;
                while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (++spins >= kWaitSpins) {
                        atomicOr(&hd->error, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        const int ntiles = P.tiles_x * P.tiles_y;
        const int t0 = (int)chunk * kChunkTiles;
        const int t1 = min(t0 + kChunkTiles, ntiles);
        for (int tt = t0; tt < t1; ++tt) {
            const int ty = tt / P.tiles_x;
            const int tx = tt - ty * P.tiles_x;
            tile_body<kForward, kCdf97, T, SPLIT, NW, K>(P, tx, ty, bufT, bufS, lane, wv);
            __syncthreads();                      // LDS edge buffers are reused by the next tile
        }
        // publish: every thread's stores before the counter update
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&done[l * count + i], (uint32_t)(t1 - t0));
    }
}

template <typename T, bool SPLIT, int NW, int K>
hipError_t launch_batched_shape(const dwt2_image* dev_imgs, int count, int levels, void* ws, uint32_t tickets,
                                hipStream_t s) {
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    static int grid_cache[16] = {0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int& grid_full = grid_cache[dev & 15];
    if (grid_full == 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_fwd_kernel<T, SPLIT, NW, K>,
                                                         NW * kLanes, 0);
        if (e != hipSuccess) return e;
        grid_full = cus * (per_cu > 0 ? per_cu : 1);
    }
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_imgs, count, levels, kCoreBY,
                       (int)sizeof(T), static_cast<unsigned char*>(ws));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = (int)(tickets < (uint32_t)grid_full ? tickets : (uint32_t)grid_full);
    hipLaunchKernelGGL((batched_fwd_kernel<T, SPLIT, NW, K>), dim3(grid), dim3(NW * kLanes), 0, s, dev_imgs, count,
                       levels, static_cast<unsigned char*>(ws));
    return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t launch_batched_cfg(int cfg, const dwt2_image* d, int count, int levels, void* ws, uint32_t tickets,
                              hipStream_t s) {
    switch (cfg) {
        case 0: return launch_batched_shape<T, SPLIT, kConfigs[0].waves, kConfigs[0].rows>(d, count, levels, ws, tickets, s);
        case 1: return launch_batched_shape<T, SPLIT, kConfigs[1].waves, kConfigs[1].rows>(d, count, levels, ws, tickets, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_batched_t(bool split, int cfg, const dwt2_image* d, int count, int levels, void* ws,
                            uint32_t tickets, hipStream_t s) {
    return split ? launch_batched_cfg<T, true>(cfg, d, count, levels, ws, tickets, s)
                 : launch_batched_cfg<T, false>(cfg, d, count, levels, ws, tickets, s);
}

}  // namespace
}  // namespace kern

bool batched_config_supported(int cfg) { return cfg == 0 || cfg == 1; }

hipError_t launch_fwd_batched(Dtype dt, bool split, int cfg, const dwt2_image* dev_imgs, int count, int levels,
                              void* ws, uint32_t tickets, hipStream_t s) {
    static_assert(kConfigs[0].algo == kAlgoTile && kConfigs[1].algo == kAlgoTile,
                  "batched kernels are instantiated for tile configurations 0 and 1");
    switch (dt) {
        case kF32: return kern::launch_batched_t<float>(split, cfg, dev_imgs, count, levels, ws, tickets, s);
        case kBF16: return kern::launch_batched_t<__hip_bfloat16>(split, cfg, dev_imgs, count, levels, ws, tickets, s);
        case kF16: return kern::launch_batched_t<__half>(split, cfg, dev_imgs, count, levels, ws, tickets, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dwt2
