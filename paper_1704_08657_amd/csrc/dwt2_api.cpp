// C ABI of the 2-D lifting DWT library: argument checks, level planning,
// workspace layout and kernel dispatch.  Every check runs on the host before
// the first HIP call, so an invalid call enqueues nothing.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "dwt2.h"
#include "dwt2_batch_plan.h"
#include "dwt2_internal.h"

static_assert(DWT2_NUM_KERNEL_CONFIGS == dwt2::kNumConfigs, "kernel configuration count in dwt2.h");

namespace {

thread_local std::string g_last_hip_error;

size_t elem_size(int dt) {
    switch (dt) {
        case DWT2_F32: return 4;
        case DWT2_BF16: return 2;
        case DWT2_F16: return 2;
        case DWT2_I32: return 4;
    }
    return 0;
}

constexpr int32_t kMaxSide = 1 << 30;
constexpr int64_t kWsAlign = 256;            // bytes; also the LL pitch granule

int64_t ws_pitch(int32_t w) {                // elements, multiple of 64
    return ((int64_t)w + 63) / 64 * 64;
}

struct Plan {
    int levels;
    int32_t h[32], w[32];                    // size transformed at each level
};

int max_levels(int32_t h, int32_t w) {
    if (h < 2 || w < 2) return 0;
    int n = 0;
    while (h >= 2 && w >= 2) {
        ++n;
        h = (h + 1) / 2;
        w = (w + 1) / 2;
    }
    return n;
}

void plan_levels(int32_t h, int32_t w, int levels, Plan* p) {
    p->levels = levels;
    for (int l = 0; l < levels; ++l) {
        p->h[l] = h;
        p->w[l] = w;
        h = (h + 1) / 2;
        w = (w + 1) / 2;
    }
}

// Two ping-pong buffers per plane for intermediate LL bands: buffer A holds
// the LL of levels 1, 3, 5, ... (largest: level 1), buffer B of levels 2,
// 4, ...  All planes' A buffers come first (plane stride a), then all B
// buffers (plane stride b); a and b are multiples of kWsAlign bytes.
struct WsLayout {
    size_t a, b;        // bytes of one plane's buffer A / B
    size_t off_b;       // offset of the B region
    size_t total;
};

WsLayout ws_layout(const Plan& p, size_t es, int32_t planes) {
    size_t a = 0, b = 0;
    for (int l = 0; l + 1 < p.levels; ++l) {  // LL of level l+1 (0-based l) is kept
        const int32_t he = (p.h[l] + 1) / 2, we = (p.w[l] + 1) / 2;
        const size_t sz = (size_t)he * (size_t)ws_pitch(we) * es;
        if (l % 2 == 0) a = a > sz ? a : sz; else b = b > sz ? b : sz;
    }
    WsLayout L;
    L.a = (a + kWsAlign - 1) / kWsAlign * kWsAlign;
    L.b = (b + kWsAlign - 1) / kWsAlign * kWsAlign;
    L.off_b = L.a * (size_t)planes;
    L.total = L.off_b + L.b * (size_t)planes;
    return L;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!na || !nb) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t span_bytes(int32_t h, int32_t w, int64_t pitch, size_t es) {
    return ((size_t)(h - 1) * (size_t)pitch + (size_t)w) * es;
}

// Bytes from the first to the last element of `planes` planes.
size_t planes_span_bytes(int32_t planes, int64_t plane_stride, int32_t h, int32_t w, int64_t pitch, size_t es) {
    return (size_t)(planes - 1) * (size_t)plane_stride * es + span_bytes(h, w, pitch, es);
}

// Every tile of a batched call runs in the same launch as the tiles of the
// other images, so no image's destination may overlap another image's
// destination or any image's source (sources may share memory: they are only
// read).  The destination spans are sorted by start; once they are known to
// be disjoint they are also sorted by end, so the only destination that can
// overlap a source [a, b) is the last one starting before b.
bool batch_spans_alias(const dwt2_image* imgs, int count, size_t es) {
    std::vector<std::pair<uintptr_t, uintptr_t>> dst((size_t)count);
    for (int i = 0; i < count; ++i) {
        const uintptr_t a = (uintptr_t)imgs[i].dst;
        dst[(size_t)i] = {a, a + span_bytes(imgs[i].height, imgs[i].width, imgs[i].dst_pitch, es)};
    }
    std::sort(dst.begin(), dst.end());
    for (size_t i = 1; i < dst.size(); ++i)
        if (dst[i].first < dst[i - 1].second) return true;
    for (int i = 0; i < count; ++i) {
        const uintptr_t a = (uintptr_t)imgs[i].src;
        const uintptr_t b = a + span_bytes(imgs[i].height, imgs[i].width, imgs[i].src_pitch, es);
        auto it = std::lower_bound(dst.begin(), dst.end(), std::make_pair(b, (uintptr_t)0));
        if (it != dst.begin() && std::prev(it)->second > a) return true;
    }
    return false;
}

// Kernel configuration selected by the flags (0 in the field = the default:
// the LDS-plane kernel for DD 13/7 and the polyconvolution, which only it
// runs; the register tile kernel otherwise).
int config_of(unsigned flags, int wavelet) {
    const unsigned t = (flags & DWT2_FLAG_KERNEL_MASK) >> DWT2_FLAG_KERNEL_SHIFT;
    if (t != 0) return (int)t - 1;
    return (wavelet == DWT2_DD137 || (flags & DWT2_FLAG_POLYCONV)) ? dwt2::kDefaultLdsConfig : dwt2::kDefaultConfig;
}

// Lifting scheme of a call.  Without a scheme flag: the fused steps,
// evaluated directly (T_P, S_U) for 4-byte samples, and for BF16 / FP16
// storage on the tile configurations as their two 1-D factors in registers
// (the same steps and barriers, 8 instead of 11 operations per block and
// step): with half the bytes per pixel that kernel is bound by its
// arithmetic.  DWT2_FLAG_FUSED asks for the direct evaluation everywhere.
dwt2::Scheme scheme_of(unsigned flags, int dtype, int wavelet, bool adjoint) {
    if (flags & DWT2_FLAG_SPLIT) return dwt2::kSchemeSplit;
    if (flags & DWT2_FLAG_SEPARABLE) return dwt2::kSchemeSeparable;
    if (flags & DWT2_FLAG_FACTORED) return dwt2::kSchemeFactored;
    if (flags & DWT2_FLAG_POLYCONV) return dwt2::kSchemePolyconv;
    if (flags & DWT2_FLAG_FUSED) return dwt2::kSchemeFused;
    const bool half = dtype == DWT2_BF16 || dtype == DWT2_F16;
    if (half && !adjoint && (wavelet == DWT2_CDF97 || wavelet == DWT2_CDF53) &&
        dwt2::kConfigs[config_of(flags, wavelet)].algo == dwt2::kAlgoTile)
        return dwt2::kSchemeFactored;
    return dwt2::kSchemeFused;
}

// The persistent forward (DWT2_FLAG_PERSISTENT: every level in one launch)
// runs CDF 9/7 with the fused or split steps on the tile configurations, for
// plane stacks of at most kMaxPersistPlanes planes.
constexpr int32_t kMaxPersistPlanes = 65536;

bool persistent_ok(int wavelet, int dtype, unsigned flags, int32_t planes) {
    return wavelet == DWT2_CDF97 && dtype != DWT2_I32 && planes <= kMaxPersistPlanes &&
           !(flags & (DWT2_FLAG_SEPARABLE | DWT2_FLAG_POLYCONV)) &&
           dwt2::persist_config_supported(config_of(flags, wavelet));
}

// Chunks and tiles of one image over all levels, for tile configuration cfg.
void image_work(int32_t h, int32_t w, int levels, int cfg, uint64_t* chunks, uint64_t* tiles) {
    const dwt2::KernelConfig c = dwt2::kConfigs[cfg];
    *chunks = 0;
    *tiles = 0;
    for (int l = 0; l < levels; ++l) {
        int32_t hl, wl, tx, ty;
        dwt2::level_size(h, w, l, &hl, &wl);
        dwt2::level_tiles(hl, wl, dwt2::core_cols(c), dwt2::core_rows(c), &tx, &ty);
        *chunks += (uint64_t)dwt2::chunk_count(ty);
        *tiles += (uint64_t)tx * (uint64_t)ty;
    }
}

// Workspace of a persistent call on `count` images (a plane stack when
// imgs == nullptr: `count` planes of h x w): the work tables and every
// image's LL bands.  The tables depend on the tile shape, so the size is the
// largest over the tile configurations.
size_t persist_bytes(const dwt2_image* imgs, int count, int32_t h, int32_t w, int levels, size_t es) {
    size_t tables = 0;
    for (int cfg = 0; cfg < dwt2::kNumConfigs; ++cfg) {
        if (!dwt2::persist_config_supported(cfg)) continue;
        uint64_t chunks = 0;
        for (int i = 0; i < (imgs ? count : 1); ++i) {
            uint64_t c, t;
            image_work(imgs ? imgs[i].height : h, imgs ? imgs[i].width : w, levels, cfg, &c, &t);
            chunks += imgs ? c : c * (uint64_t)count;
        }
        const size_t off = dwt2::batch_layout(count, levels, chunks).off_ll;
        tables = tables > off ? tables : off;
    }
    size_t ll = 0;
    if (imgs)
        for (int i = 0; i < count; ++i) ll += dwt2::image_ll_bytes(imgs[i].height, imgs[i].width, levels, es);
    else
        ll = (size_t)count * dwt2::image_ll_bytes(h, w, levels, es);
    return tables + ll;
}

int validate(const void* src, void* dst, int32_t planes, int64_t sps, int64_t dps, int32_t h, int32_t w,
             int64_t sp, int64_t dp, int dtype, int wavelet, int levels, int boundary, unsigned flags,
             const void* ws, size_t ws_bytes, bool adjoint, bool own_ws = false) {
    if (!src || !dst) return DWT2_E_NULL;
    if (planes < 1) return DWT2_E_COUNT;
    if (wavelet != DWT2_CDF97 && wavelet != DWT2_CDF53_REV && wavelet != DWT2_CDF53 && wavelet != DWT2_DD137)
        return DWT2_E_WAVELET;
    if (dtype != DWT2_F32 && dtype != DWT2_BF16 && dtype != DWT2_F16 && dtype != DWT2_I32)
        return DWT2_E_DTYPE;
    if ((wavelet == DWT2_CDF53_REV) != (dtype == DWT2_I32)) return DWT2_E_DTYPE;
    if (boundary != DWT2_SYMMETRIC_WHOLE) return DWT2_E_BOUNDARY;
    if (flags & ~(DWT2_FLAG_SPLIT | DWT2_FLAG_SEPARABLE | DWT2_FLAG_FACTORED | DWT2_FLAG_POLYCONV |
                  DWT2_FLAG_FUSED | DWT2_FLAG_PERSISTENT | DWT2_FLAG_KERNEL_MASK))
        return DWT2_E_FLAGS;
    if (((flags & DWT2_FLAG_KERNEL_MASK) >> DWT2_FLAG_KERNEL_SHIFT) > (unsigned)dwt2::kNumConfigs)
        return DWT2_E_FLAGS;
    if (adjoint && wavelet != DWT2_CDF97) return DWT2_E_WAVELET;
    if ((flags & DWT2_FLAG_SPLIT) && (wavelet == DWT2_CDF53_REV || adjoint)) return DWT2_E_FLAGS;
    // at most one scheme flag; the separable and factored schemes: forward /
    // inverse on tile configurations (the separable one also on LDS-plane
    // configurations); the polyconvolution: CDF 9/7 forward / inverse on
    // LDS-plane configurations
    const unsigned schemes =
        flags & (DWT2_FLAG_SPLIT | DWT2_FLAG_SEPARABLE | DWT2_FLAG_FACTORED | DWT2_FLAG_POLYCONV | DWT2_FLAG_FUSED);
    if (schemes & (schemes - 1)) return DWT2_E_FLAGS;
    const int algo = dwt2::kConfigs[config_of(flags, wavelet)].algo;
    if ((flags & (DWT2_FLAG_SEPARABLE | DWT2_FLAG_FACTORED)) && (adjoint || algo == dwt2::kAlgoStream))
        return DWT2_E_FLAGS;
    if ((flags & DWT2_FLAG_POLYCONV) && wavelet != DWT2_CDF97) return DWT2_E_FLAGS;
    if ((flags & DWT2_FLAG_PERSISTENT) && (adjoint || !persistent_ok(wavelet, dtype, flags, planes)))
        return DWT2_E_FLAGS;
    // the LDS-plane kernel: float wavelets, forward / inverse, fused,
    // separable and polyconvolution schemes; it alone runs DD 13/7 and the
    // polyconvolution
    if (algo == dwt2::kAlgoLds &&
        (adjoint || wavelet == DWT2_CDF53_REV || (flags & (DWT2_FLAG_SPLIT | DWT2_FLAG_FACTORED))))
        return DWT2_E_FLAGS;
    if (algo != dwt2::kAlgoLds && (wavelet == DWT2_DD137 || (flags & DWT2_FLAG_POLYCONV))) return DWT2_E_FLAGS;
    if (h < 2 || w < 2 || h > kMaxSide || w > kMaxSide) return DWT2_E_SHAPE;
    if (sp < w || dp < w) return DWT2_E_PITCH;
    // planes of one buffer must not overlap
    const int64_t plane_elems = (int64_t)(h - 1) * sp + w, plane_elems_d = (int64_t)(h - 1) * dp + w;
    if (planes > 1 && (sps < plane_elems || dps < plane_elems_d)) return DWT2_E_PITCH;
    if (levels < 1 || levels > max_levels(h, w)) return DWT2_E_LEVELS;
    size_t need = 0;
    dwt2_workspace_bytes_planes(h, w, levels, (dwt2_dtype)dtype, planes, &need);
    // own_ws: the workspace is the library's scratch array (checked by the caller)
    if (need > 0 && !own_ws && (!ws || ws_bytes < need)) return DWT2_E_WORKSPACE;
    const size_t es = elem_size(dtype);
    const size_t ns = planes_span_bytes(planes, sps, h, w, sp, es), nd = planes_span_bytes(planes, dps, h, w, dp, es);
    if (ranges_overlap(src, ns, dst, nd)) return DWT2_E_ALIAS;
    if (need > 0 && !own_ws && (ranges_overlap(ws, need, src, ns) || ranges_overlap(ws, need, dst, nd)))
        return DWT2_E_ALIAS;
    return DWT2_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int report(hipError_t e) {
    if (e == hipSuccess) return DWT2_OK;
    g_last_hip_error = hipGetErrorString(e);
    return DWT2_E_HIP;
}

dwt2::Dtype to_dtype(int d) { return (dwt2::Dtype)d; }
dwt2::Wavelet to_wav(int w) {
    return w == DWT2_CDF97 ? dwt2::kCdf97 : w == DWT2_CDF53 ? dwt2::kCdf53Real : w == DWT2_DD137 ? dwt2::kDd137
                                                                                                  : dwt2::kCdf53;
}

// Work-group grid of one level for kernel configuration `cfg`.
void plan_grid(int cfg, dwt2::LevelParams* lp) {
    const dwt2::KernelConfig c = dwt2::kConfigs[cfg];
    const int32_t nEr = (lp->h + 1) / 2, nEc = (lp->w + 1) / 2;
    if (c.algo != dwt2::kAlgoStream) {
        const int cy = dwt2::core_rows(c);
        const int cx = dwt2::core_cols(c);
        lp->tiles_x = (nEc + cx - 1) / cx;
        lp->tiles_y = (nEr + cy - 1) / cy;
        lp->seg_rows = 0;
    } else {
        const int32_t strips = (nEc + dwt2::kStreamCoreBX - 1) / dwt2::kStreamCoreBX;
        lp->tiles_x = (strips + c.waves - 1) / c.waves;
        lp->tiles_y = (nEr + c.seg - 1) / c.seg;
        lp->seg_rows = c.seg;
    }
}

// Launch one level for every plane, in grid chunks of at most
// kMaxGridPlanes planes.
int launch_planes(dwt2::Direction dir, int wavelet, int dtype, unsigned flags, dwt2::LevelParams lp,
                  int32_t planes, size_t es, hipStream_t s) {
    for (int32_t p0 = 0; p0 < planes; p0 += dwt2::kMaxGridPlanes) {
        const int32_t n = planes - p0 < dwt2::kMaxGridPlanes ? planes - p0 : dwt2::kMaxGridPlanes;
        dwt2::LevelParams q = lp;
        if (p0 > 0) {
            q.in = lp.in ? (const char*)lp.in + (size_t)p0 * (size_t)lp.in_ps * es : nullptr;
            q.in_ll = lp.in_ll ? (const char*)lp.in_ll + (size_t)p0 * (size_t)lp.in_ll_ps * es : nullptr;
            q.out = lp.out ? (char*)lp.out + (size_t)p0 * (size_t)lp.out_ps * es : nullptr;
            q.out_ll = lp.out_ll ? (char*)lp.out_ll + (size_t)p0 * (size_t)lp.out_ll_ps * es : nullptr;
        }
        const int rc = report(dwt2::launch_level(dir, to_wav(wavelet), to_dtype(dtype),
                                                 scheme_of(flags, dtype, wavelet, dir == dwt2::kAdjoint),
                                                 config_of(flags, wavelet), q, n, s));
        if (rc) return rc;
    }
    return DWT2_OK;
}

// Vector access needs every plane's row bases aligned: the plane strides
// (unused when there is one plane) as well as the pitches.
bool stride_ok(int32_t planes, int64_t stride, int v) { return planes == 1 || stride % v == 0; }

// Forward: level l reads the LL of level l-1 (src for l = 0) and writes its
// details into dst at the level's region origin (dst itself: every level's
// region starts at (0, 0)), its LL into the workspace or, for the last level,
// into dst.
// Whether a level stores the output the next level of the call reads with
// ordinary stores (LevelParams::ll_cached): measured on MI355X, it pays for
// outputs of 32 MiB and more (an 8192^2 FP32 level's LL band: +4% on two
// levels, forward and inverse) and costs 2% on smaller ones (4096^2, whose
// LL band the nontemporal path leaves in the Infinity Cache anyway).
bool cached_output(int32_t planes, int32_t h, int32_t w, size_t es) {
    return (uint64_t)planes * (uint64_t)h * (uint64_t)w * es >= ((uint64_t)32 << 20);
}

int run_forward(const void* src, void* dst, int32_t planes, int64_t sps, int64_t dps, int32_t h, int32_t w,
                int64_t sp, int64_t dp, int dtype, int wavelet, int levels, unsigned flags, void* ws,
                hipStream_t s) {
    // one level is one launch either way (and needs no workspace)
    if ((flags & DWT2_FLAG_PERSISTENT) && levels > 1) {
        const int cfg = config_of(flags, wavelet);
        uint64_t chunks, tiles;
        image_work(h, w, levels, cfg, &chunks, &tiles);
        const dwt2::ImageSet S{nullptr, src, dst, sps, dps, sp, dp, h, w};
        const dwt2::BatchLayout L = dwt2::batch_layout(planes, levels, chunks * (uint64_t)planes);
        return report(dwt2::launch_fwd_persistent(to_dtype(dtype), scheme_of(flags, dtype, wavelet, false), cfg, S,
                                                  planes, levels, ws, L, tiles * (uint64_t)planes, s));
    }
    Plan p;
    plan_levels(h, w, levels, &p);
    const size_t es = elem_size(dtype);
    const WsLayout L = ws_layout(p, es, planes);
    char* bufs[2] = {(char*)ws, (char*)ws + L.off_b};
    const int64_t buf_ps[2] = {(int64_t)(L.a / es), (int64_t)(L.b / es)};
    const void* in = src;
    int64_t in_pitch = sp, in_ps = sps;
    for (int l = 0; l < levels; ++l) {
        dwt2::LevelParams lp{};
        lp.h = p.h[l];
        lp.w = p.w[l];
        lp.in = in;
        lp.in_pitch = in_pitch;
        lp.in_ps = in_ps;
        lp.out = dst;
        lp.out_pitch = dp;
        lp.out_ps = dps;
        const bool last = l + 1 == levels;
        lp.ll_cached = !last && cached_output(planes, (lp.h + 1) / 2, (lp.w + 1) / 2, es) ? 1 : 0;
        lp.out_ll = last ? dst : (void*)bufs[l % 2];
        lp.out_ll_pitch = last ? dp : ws_pitch((lp.w + 1) / 2);
        lp.out_ll_ps = last ? dps : buf_ps[l % 2];
        plan_grid(config_of(flags, wavelet), &lp);
        const int32_t nEc = (lp.w + 1) / 2;
        const int sv = dwt2::subband_vec(dwt2::kConfigs[config_of(flags, wavelet)]);
        lp.vec = aligned(lp.in, 4 * es) && lp.in_pitch % 4 == 0 && stride_ok(planes, lp.in_ps, 4) &&
                 aligned(lp.out, sv * es) && lp.out_pitch % sv == 0 && stride_ok(planes, lp.out_ps, sv) &&
                 nEc % sv == 0 && aligned(lp.out_ll, sv * es) && lp.out_ll_pitch % sv == 0 &&
                 stride_ok(planes, lp.out_ll_ps, sv);
        // sample pairs: every row base (and plane stride) 8-byte aligned
        lp.vec8 = aligned(lp.in, 2 * es) && lp.in_pitch % 2 == 0 && stride_ok(planes, lp.in_ps, 2) &&
                  aligned(lp.out, 2 * es) && lp.out_pitch % 2 == 0 && stride_ok(planes, lp.out_ps, 2) &&
                  aligned(lp.out_ll, 2 * es) && lp.out_ll_pitch % 2 == 0 && stride_ok(planes, lp.out_ll_ps, 2);
        // image rows 16-byte aligned
        const int v16 = (int)(16 / es);
        lp.vec16 = aligned(lp.in, 16) && lp.in_pitch % v16 == 0 && stride_ok(planes, lp.in_ps, v16);
        const int rc = launch_planes(dwt2::kForward, wavelet, dtype, flags, lp, planes, es, s);
        if (rc) return rc;
        in = lp.out_ll;
        in_pitch = lp.out_ll_pitch;
        in_ps = lp.out_ll_ps;
    }
    return DWT2_OK;
}

// Inverse / adjoint: coarsest level first.  Level l reads its LL (src for the
// coarsest level, else the workspace written by level l+1) and its details
// from src, and writes its image into the workspace or, for l = 0, into dst.
int run_backward(dwt2::Direction dir, const void* src, void* dst, int32_t planes, int64_t sps, int64_t dps,
                 int32_t h, int32_t w, int64_t sp, int64_t dp, int dtype, int wavelet, int levels,
                 unsigned flags, void* ws, hipStream_t s) {
    Plan p;
    plan_levels(h, w, levels, &p);
    const size_t es = elem_size(dtype);
    const WsLayout L = ws_layout(p, es, planes);
    char* bufs[2] = {(char*)ws, (char*)ws + L.off_b};
    const int64_t buf_ps[2] = {(int64_t)(L.a / es), (int64_t)(L.b / es)};
    const void* ll = src;
    int64_t ll_pitch = sp, ll_ps = sps;
    for (int l = levels - 1; l >= 0; --l) {
        dwt2::LevelParams lp{};
        lp.h = p.h[l];
        lp.w = p.w[l];
        lp.in = src;
        lp.in_pitch = sp;
        lp.in_ps = sps;
        lp.in_ll = ll;
        lp.in_ll_pitch = ll_pitch;
        lp.in_ll_ps = ll_ps;
        // the image of level l is the LL of level l-1 (kept in buffer (l-1) % 2)
        lp.ll_cached = l > 0 && cached_output(planes, p.h[l], p.w[l], es) ? 1 : 0;
        lp.out = l == 0 ? dst : (void*)bufs[(l - 1) % 2];
        lp.out_pitch = l == 0 ? dp : ws_pitch(lp.w);
        lp.out_ps = l == 0 ? dps : buf_ps[(l - 1) % 2];
        plan_grid(config_of(flags, wavelet), &lp);
        const int32_t nEc = (lp.w + 1) / 2;
        const int sv = dwt2::subband_vec(dwt2::kConfigs[config_of(flags, wavelet)]);
        lp.vec = aligned(lp.in, sv * es) && lp.in_pitch % sv == 0 && stride_ok(planes, lp.in_ps, sv) &&
                 nEc % sv == 0 && aligned(lp.in_ll, sv * es) && lp.in_ll_pitch % sv == 0 &&
                 stride_ok(planes, lp.in_ll_ps, sv) && aligned(lp.out, 4 * es) && lp.out_pitch % 4 == 0 &&
                 stride_ok(planes, lp.out_ps, 4);
        // sample pairs: every row base (and plane stride) 8-byte aligned
        lp.vec8 = aligned(lp.in, 2 * es) && lp.in_pitch % 2 == 0 && stride_ok(planes, lp.in_ps, 2) &&
                  aligned(lp.in_ll, 2 * es) && lp.in_ll_pitch % 2 == 0 && stride_ok(planes, lp.in_ll_ps, 2) &&
                  aligned(lp.out, 2 * es) && lp.out_pitch % 2 == 0 && stride_ok(planes, lp.out_ps, 2);
        // image rows 16-byte aligned
        const int v16 = (int)(16 / es);
        lp.vec16 = aligned(lp.out, 16) && lp.out_pitch % v16 == 0 && stride_ok(planes, lp.out_ps, v16);
        const int rc = launch_planes(dir, wavelet, dtype, flags, lp, planes, es, s);
        if (rc) return rc;
        ll = lp.out;
        ll_pitch = lp.out_pitch;
        ll_ps = lp.out_ps;
    }
    return DWT2_OK;
}

// Workspace of dwt2_fwd_noalloc: one fixed array per GPU (the code object
// holds it on every device it is loaded on, until the process ends).  Host
// code must not pass `scratch` itself to a kernel or a copy: in host code the
// name is a host-side stand-in, not the device address.  The device address
// is looked up once per device (hipGetSymbolAddress with that device
// current) and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DWT2_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(e);
    if (dev < 0 || dev >= kMaxDevices) return report(hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return report(e);
        if (!p) return report(hipErrorInvalidSymbol);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DWT2_OK;
}

}  // namespace

extern "C" {

int dwt2_max_levels(int32_t height, int32_t width) { return max_levels(height, width); }

int dwt2_workspace_bytes_planes(int32_t height, int32_t width, int levels, dwt2_dtype dtype, int32_t planes,
                                size_t* bytes) {
    if (!bytes) return DWT2_E_NULL;
    *bytes = 0;
    const size_t es = elem_size(dtype);
    if (!es) return DWT2_E_DTYPE;
    if (planes < 1) return DWT2_E_COUNT;
    if (height < 2 || width < 2 || height > kMaxSide || width > kMaxSide) return DWT2_E_SHAPE;
    if (levels < 1 || levels > max_levels(height, width)) return DWT2_E_LEVELS;
    Plan p;
    plan_levels(height, width, levels, &p);
    size_t n = ws_layout(p, es, planes).total;
    // a float multi-level forward may take the persistent path
    if (levels > 1 && dtype != DWT2_I32 && planes <= kMaxPersistPlanes) {
        const size_t q = persist_bytes(nullptr, planes, height, width, levels, es);
        n = n > q ? n : q;
    }
    *bytes = n;
    return DWT2_OK;
}

int dwt2_workspace_bytes(int32_t height, int32_t width, int levels, dwt2_dtype dtype, size_t* bytes) {
    return dwt2_workspace_bytes_planes(height, width, levels, dtype, 1, bytes);
}

int dwt2_fwd_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride, int64_t dst_plane_stride,
                    int32_t height, int32_t width, int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
                    dwt2_wavelet wavelet, int levels, dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream) {
    const int rc = validate(src, dst, planes, src_plane_stride, dst_plane_stride, height, width, src_pitch,
                            dst_pitch, dtype, wavelet, levels, boundary, flags, workspace, workspace_bytes, false);
    if (rc) return rc;
    return run_forward(src, dst, planes, src_plane_stride, dst_plane_stride, height, width, src_pitch, dst_pitch,
                       dtype, wavelet, levels, flags, workspace, (hipStream_t)stream);
}

int dwt2_inv_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride, int64_t dst_plane_stride,
                    int32_t height, int32_t width, int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
                    dwt2_wavelet wavelet, int levels, dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream) {
    if (flags & DWT2_FLAG_PERSISTENT) return DWT2_E_FLAGS;   // a forward-only path
    const int rc = validate(src, dst, planes, src_plane_stride, dst_plane_stride, height, width, src_pitch,
                            dst_pitch, dtype, wavelet, levels, boundary, flags, workspace, workspace_bytes, false);
    if (rc) return rc;
    return run_backward(dwt2::kInverse, src, dst, planes, src_plane_stride, dst_plane_stride, height, width,
                        src_pitch, dst_pitch, dtype, wavelet, levels, flags, workspace, (hipStream_t)stream);
}

int dwt2_adj_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride, int64_t dst_plane_stride,
                    int32_t height, int32_t width, int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
                    dwt2_wavelet wavelet, int levels, dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream) {
    const int rc = validate(src, dst, planes, src_plane_stride, dst_plane_stride, height, width, src_pitch,
                            dst_pitch, dtype, wavelet, levels, boundary, flags, workspace, workspace_bytes, true);
    if (rc) return rc;
    return run_backward(dwt2::kAdjoint, src, dst, planes, src_plane_stride, dst_plane_stride, height, width,
                        src_pitch, dst_pitch, dtype, wavelet, levels, flags, workspace, (hipStream_t)stream);
}

int dwt2_fwd(const void* src, void* dst, int32_t height, int32_t width, int64_t src_pitch,
             int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
             dwt2_boundary boundary, unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream) {
    return dwt2_fwd_planes(src, dst, 1, 0, 0, height, width, src_pitch, dst_pitch, dtype, wavelet, levels, boundary,
                           flags, workspace, workspace_bytes, stream);
}

int dwt2_inv(const void* src, void* dst, int32_t height, int32_t width, int64_t src_pitch,
             int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
             dwt2_boundary boundary, unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream) {
    return dwt2_inv_planes(src, dst, 1, 0, 0, height, width, src_pitch, dst_pitch, dtype, wavelet, levels, boundary,
                           flags, workspace, workspace_bytes, stream);
}

int dwt2_adj(const void* src, void* dst, int32_t height, int32_t width, int64_t src_pitch,
             int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
             dwt2_boundary boundary, unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream) {
    return dwt2_adj_planes(src, dst, 1, 0, 0, height, width, src_pitch, dst_pitch, dtype, wavelet, levels, boundary,
                           flags, workspace, workspace_bytes, stream);
}

int dwt2_fwd_noalloc(const void* src, void* dst, int32_t height, int32_t width, int64_t src_pitch,
                     int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
                     dwt2_boundary boundary, unsigned flags, void* stream) {
    int rc = validate(src, dst, 1, 0, 0, height, width, src_pitch, dst_pitch, dtype, wavelet, levels, boundary,
                      flags, nullptr, 0, false, /*own_ws=*/true);
    if (rc) return rc;
    size_t need = 0;
    rc = dwt2_workspace_bytes(height, width, levels, dtype, &need);
    if (rc) return rc;
    if (need > DWT2_SCRATCH_BYTES) return DWT2_E_SCRATCH;
    void* ws = nullptr;
    if (need > 0) {                 // one level needs no workspace
        rc = scratch_address(&ws);
        if (rc) return rc;
    }
    return run_forward(src, dst, 1, 0, 0, height, width, src_pitch, dst_pitch, dtype, wavelet, levels, flags, ws,
                       (hipStream_t)stream);
}

int dwt2_kernel_config(int index, int* algorithm, int* waves, int* rows, int* core_cols, int* core_rows) {
    if (index < 0 || index >= dwt2::kNumConfigs) return DWT2_E_FLAGS;
    const dwt2::KernelConfig c = dwt2::kConfigs[index];
    if (algorithm) *algorithm = c.algo;
    if (waves) *waves = c.waves;
    if (rows) *rows = c.rows;
    if (core_cols) *core_cols = c.algo != dwt2::kAlgoStream ? dwt2::core_cols(c) : dwt2::kStreamCoreBX;
    if (core_rows) *core_rows = c.algo != dwt2::kAlgoStream ? dwt2::core_rows(c) : c.seg;
    return DWT2_OK;
}

int dwt2_workspace_bytes_batched(const dwt2_image* images, int count, dwt2_dtype dtype, int levels,
                                 size_t* bytes) {
    if (!bytes || !images) return DWT2_E_NULL;
    *bytes = 0;
    if (count < 1) return DWT2_E_COUNT;
    const size_t es = elem_size(dtype);
    if (!es) return DWT2_E_DTYPE;
    for (int i = 0; i < count; ++i) {
        const dwt2_image& im = images[i];
        if (im.height < 2 || im.width < 2 || im.height > kMaxSide || im.width > kMaxSide) return DWT2_E_SHAPE;
        if (levels < 1 || levels > max_levels(im.height, im.width)) return DWT2_E_LEVELS;
    }
    // one launch per level: tile tables and ping-pong LL buffers; the
    // persistent launch: work tables and one LL band per level
    const dwt2::LevelBatchLayout L = dwt2::level_batch_layout(count, levels);
    size_t n = L.off_ll;
    for (int i = 0; i < count; ++i) n += dwt2::pingpong_ll_bytes(images[i].height, images[i].width, levels, es);
    const size_t q = persist_bytes(images, count, 0, 0, levels, es);
    *bytes = n > q ? n : q;
    return DWT2_OK;
}

int dwt2_fwd_batched(const dwt2_image* host_images, const dwt2_image* device_images, int count,
                     dwt2_dtype dtype, dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
                     unsigned flags, void* workspace, size_t workspace_bytes, void* stream) {
    if (!host_images || !device_images || !workspace) return DWT2_E_NULL;
    if (count < 1) return DWT2_E_COUNT;
    if (wavelet != DWT2_CDF97) return DWT2_E_WAVELET;        // batched path: CDF 9/7
    if (dtype != DWT2_F32 && dtype != DWT2_BF16 && dtype != DWT2_F16) return DWT2_E_DTYPE;
    if (boundary != DWT2_SYMMETRIC_WHOLE) return DWT2_E_BOUNDARY;
    if (flags & ~(DWT2_FLAG_SPLIT | DWT2_FLAG_FACTORED | DWT2_FLAG_FUSED | DWT2_FLAG_PERSISTENT |
                  DWT2_FLAG_KERNEL_MASK))
        return DWT2_E_FLAGS;
    {
        const unsigned sch = flags & (DWT2_FLAG_SPLIT | DWT2_FLAG_FACTORED | DWT2_FLAG_FUSED);
        if (sch & (sch - 1)) return DWT2_E_FLAGS;          // at most one scheme
    }
    if (((flags & DWT2_FLAG_KERNEL_MASK) >> DWT2_FLAG_KERNEL_SHIFT) > (unsigned)dwt2::kNumConfigs)
        return DWT2_E_FLAGS;
    const int cfg = config_of(flags, wavelet);
    if (!dwt2::persist_config_supported(cfg)) return DWT2_E_FLAGS;
    const size_t es = elem_size(dtype);
    const dwt2::KernelConfig kc = dwt2::kConfigs[cfg];
    uint64_t tiles[32] = {0}, chunks = 0, all_tiles = 0;
    for (int i = 0; i < count; ++i) {
        const dwt2_image& im = host_images[i];
        if (!im.src || !im.dst) return DWT2_E_NULL;
        if (im.height < 2 || im.width < 2 || im.height > kMaxSide || im.width > kMaxSide) return DWT2_E_SHAPE;
        if (im.src_pitch < im.width || im.dst_pitch < im.width) return DWT2_E_PITCH;
        if (levels < 1 || levels > max_levels(im.height, im.width)) return DWT2_E_LEVELS;
        if (ranges_overlap(im.src, span_bytes(im.height, im.width, im.src_pitch, es), im.dst,
                           span_bytes(im.height, im.width, im.dst_pitch, es)))
            return DWT2_E_ALIAS;
        for (int l = 0; l < levels; ++l)
            tiles[l] += dwt2::level_tile_count(im.height, im.width, l, dwt2::core_cols(kc), dwt2::core_rows(kc));
        uint64_t c, t;
        image_work(im.height, im.width, levels, cfg, &c, &t);
        chunks += c;
        all_tiles += t;
    }
    if (batch_spans_alias(host_images, count, es)) return DWT2_E_ALIAS;
    // ticket numbers and counters are 32-bit
    for (int l = 0; l < levels; ++l)
        if (tiles[l] > 0x7fff0000ull) return DWT2_E_SHAPE;
    if (chunks > 0x7fff0000ull) return DWT2_E_SHAPE;
    size_t need = 0;
    const int st = dwt2_workspace_bytes_batched(host_images, count, dtype, levels, &need);
    if (st) return st;
    if (workspace_bytes < need) return DWT2_E_WORKSPACE;
    for (int i = 0; i < count; ++i) {
        const dwt2_image& im = host_images[i];
        if (ranges_overlap(workspace, need, im.src, span_bytes(im.height, im.width, im.src_pitch, es)) ||
            ranges_overlap(workspace, need, im.dst, span_bytes(im.height, im.width, im.dst_pitch, es)))
            return DWT2_E_ALIAS;
    }
    const dwt2::Scheme sch = scheme_of(flags, dtype, wavelet, false);
    if ((flags & DWT2_FLAG_PERSISTENT) && levels > 1) {
        const dwt2::ImageSet S{device_images, nullptr, nullptr, 0, 0, 0, 0, 0, 0};
        const dwt2::BatchLayout L = dwt2::batch_layout(count, levels, chunks);
        return report(dwt2::launch_fwd_persistent(to_dtype(dtype), sch, cfg, S, count, levels, workspace, L,
                                                  all_tiles, (hipStream_t)stream));
    }
    uint32_t tiles_per_level[32];
    for (int l = 0; l < levels; ++l) tiles_per_level[l] = (uint32_t)tiles[l];
    return report(dwt2::launch_fwd_batched_levels(to_dtype(dtype), sch, cfg, device_images, count, levels,
                                                  workspace, tiles_per_level, (hipStream_t)stream));
}

int dwt2_workspace_status(const void* header) {
    if (!header) return DWT2_E_NULL;
    return static_cast<const uint32_t*>(header)[0] != 0u ? DWT2_E_TIMEOUT : DWT2_OK;
}

const char* dwt2_status_string(int status) {
    switch (status) {
        case DWT2_OK: return "ok";
        case DWT2_E_NULL: return "null pointer";
        case DWT2_E_SHAPE: return "height and width must be in [2, 2^30]";
        case DWT2_E_LEVELS: return "level count out of range for this shape";
        case DWT2_E_DTYPE: return "dtype not valid for this wavelet";
        case DWT2_E_WAVELET: return "unknown or unsupported wavelet";
        case DWT2_E_BOUNDARY: return "unknown boundary extension";
        case DWT2_E_PITCH: return "pitch smaller than width";
        case DWT2_E_WORKSPACE: return "workspace missing or too small";
        case DWT2_E_ALIAS: return "src, dst and workspace must not overlap";
        case DWT2_E_HIP: return "HIP runtime error";
        case DWT2_E_FLAGS: return "flags not valid for this call";
        case DWT2_E_COUNT: return "image count must be positive";
        case DWT2_E_SCRATCH: return "the call needs more workspace than the library's fixed scratch array";
        case DWT2_E_TIMEOUT: return "a dependency wait of the persistent forward ran out of time: outputs invalid";
    }
    return "unknown status";
}

const char* dwt2_last_hip_error(void) { return g_last_hip_error.c_str(); }

}  // extern "C"
