// Non-separable 2-D lifting DWT kernels for AMD gfx950 (CDNA 4, wave64).
//
// Method (Barina et al., "Accelerating Discrete Wavelet Transforms on Parallel
// Architectures", Section "Proposed Schemes"): every pair of separable lifting
// steps T_P^V T_P^H and S_U^V S_U^H is fused into one spatial predict T_P and
// one spatial update S_U over the four polyphase components of 2x2 pixel
// blocks, so one scale of CDF 9/7 needs 4 barriers (not 8) and the integer
// CDF 5/3 needs 2 (not 4).  Section "Optimization Approach" (P = P0 + P1,
// U = U0 + U1, constant parts as barrier-free separable lifting) is the
// `split` variant.
//
// Mapping to gfx950 (not the paper's OpenCL or shader design):
//   * one work-group = NW wave64s = one tile of 128 x (NW * K) blocks
//     (e.g. 256 x 128 pixels for NW = K = 8) with a 2-block halo recomputed
//     on every side;
//   * each lane owns two horizontally adjacent blocks ("L" and "R") for K
//     consecutive block rows, all in VGPRs: K rows x 2 blocks x 4 components;
//   * a step reads neighbours at +1 (predict-shaped: right / down) or at -1
//     (update-shaped: left / up).  Horizontal neighbours come from the
//     adjacent lane through DPP wave shifts, vertical ones from the lane's own
//     registers, except at the boundary between two waves, where the edge row
//     is published to LDS before the step's single s_barrier (two LDS buffers,
//     one for each step shape, so one barrier per step suffices);
//   * loads are 4-pixel vectors per image row, stores are 2-block vectors per
//     subband row, both coalesced across the wave;
//   * tiles touching the image border take a path that clamps neighbour
//     indices into each component's extent (whole-point symmetric extension)
//     or, for the adjoint, applies the transposed border weights; interior
//     tiles take a branch-free path;
//   * the tile index is remapped so that consecutive tiles of the image land
//     on the same XCD (work-groups are dealt round-robin over the 8 XCDs), so
//     the halo re-reads of neighbouring tiles hit that XCD's L2.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dwt2_internal.h"

namespace dwt2 {
namespace {

// CDF 9/7 lifting factorisation (Daubechies & Sweldens): predict alpha,
// update beta, predict gamma, update delta; zeta scales low-pass outputs (and
// 1/zeta high-pass outputs) per axis so that the low-pass DC gain is sqrt(2):
// zeta = sqrt(2) / (1 + 2 beta (1 + 2 alpha)).
constexpr float kAlpha = -1.586134342059924f;
constexpr float kBeta = -0.052980118572961f;
constexpr float kGamma = 0.882911075530934f;
constexpr float kDelta = 0.443506852043971f;
constexpr double kZeta = 1.1496043988602418;
constexpr float kZeta2 = (float)(kZeta * kZeta);
constexpr float kZetaM2 = (float)(1.0 / (kZeta * kZeta));


// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------
template <typename T> struct St;
template <> struct St<float> {
    using V = float;
    __device__ static V load(float v) { return v; }
    __device__ static float store(V v) { return v; }
};
template <> struct St<__hip_bfloat16> {
    using V = float;
    __device__ static V load(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ static __hip_bfloat16 store(V v) { return __float2bfloat16(v); }
};
template <> struct St<__half> {
    using V = float;
    __device__ static V load(__half v) { return __half2float(v); }
    __device__ static __half store(V v) { return __float2half(v); }
};
template <> struct St<int32_t> {
    using V = int;
    __device__ static V load(int32_t v) { return v; }
    __device__ static int32_t store(V v) { return v; }
};

template <typename T> struct alignas(4 * sizeof(T)) Pack4 { T v[4]; };
template <typename T> struct alignas(2 * sizeof(T)) Pack2 { T v[2]; };

// ---------------------------------------------------------------------------
// cross-lane shifts (DPP, whole wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_from_right(int v) {   // lane i <- lane i+1
    return __builtin_amdgcn_update_dpp(0, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_left(int v) {    // lane i <- lane i-1
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(dpp_from_right(__float_as_int(v)));
}
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(dpp_from_left(__float_as_int(v)));
}
__device__ __forceinline__ int from_right(int v) { return dpp_from_right(v); }
__device__ __forceinline__ int from_left(int v) { return dpp_from_left(v); }

// ---------------------------------------------------------------------------
// geometry of one tile as seen by one lane
// ---------------------------------------------------------------------------
struct Geo {
    int gcL;          // global block column of the lane's L block (R = gcL + 1)
    int gr0;          // global block row of the lane's register row 0
    int nEr, nOr;     // rows of the even-row (x0, x1) / odd-row (x2, x3) components
    int nEc, nOc;     // columns of the even-col (x0, x2) / odd-col (x1, x3) components
};

// Step kinds.
enum Kind : int {
    kFloat = 0,      // fused float step (forward, inverse: coefficient sign)
    kSplitLocal = 1, // not a neighbour step (local constant part)
    kSplit = 2,      // nonlocal P1 / U1 part of the split
    kAdj = 3,        // transposed step with transposed border weights
    kIntFwd = 4,     // reversible 5/3 forward (with neighbour recomputation)
    kIntInv = 5      // reversible 5/3 inverse
};

template <typename V> struct Vec4 { V a, b, c, d; };

// ---- predict-shaped block update (reads right / down / down-right) --------
// Operands: own x0..x3; right: x0R, x2R; down: x0D, x1D; diagonal x0DR.
template <int KIND, bool EDGE, typename V>
__device__ __forceinline__ void plus_block(V& x0, V& x1, V& x2, V& x3,
                                           V x0R, V x2R, V x0D, V x1D, V x0DR,
                                           int gc, int gr, const Geo& g, float c) {
    if constexpr (KIND == kAdj) {
        // transpose of an update-shaped step: odd[k] += c (al_k e[k] + be_k e[k+1])
        // with al_k = 1 + [k == 0], be_k = [k+1 < ne] + [k+1 == no && ne > no]
        float alc = 1.f, bec = 1.f, alr = 1.f, ber = 1.f;
        if constexpr (EDGE) {
            alc = (gc == 0) ? 2.f : 1.f;
            bec = (float)((gc + 1 < g.nEc) + (gc + 1 == g.nOc && g.nEc > g.nOc));
            alr = (gr == 0) ? 2.f : 1.f;
            ber = (float)((gr + 1 < g.nEr) + (gr + 1 == g.nOr && g.nEr > g.nOr));
        }
        const float cc = c * c;
        const V h0 = fmaf(bec, x0R, alc * x0);
        const V h0d = fmaf(bec, x0DR, alc * x0D);
        x3 = fmaf(cc, fmaf(ber, h0d, alr * h0),
                  fmaf(c, fmaf(ber, x1D, alr * x1), fmaf(c, fmaf(bec, x2R, alc * x2), x3)));
        x1 = fmaf(c, h0, x1);
        x2 = fmaf(c, fmaf(ber, x0D, alr * x0), x2);
    } else {
        if constexpr (EDGE) {
            const bool cR = gc + 1 < g.nEc;
            const bool rD = gr + 1 < g.nEr;
            x0DR = rD ? (cR ? x0DR : x0D) : (cR ? x0R : x0);
            x0R = cR ? x0R : x0;
            x2R = cR ? x2R : x2;
            x0D = rD ? x0D : x0;
            x1D = rD ? x1D : x1;
        }
        if constexpr (KIND == kFloat) {
            const float cc = c * c;
            const V t0 = x0 + x0R;
            const V t1 = x0D + x0DR;
            x3 = fmaf(cc, t0 + t1, fmaf(c, x1 + x1D, fmaf(c, x2 + x2R, x3)));
            x1 = fmaf(c, t0, x1);
            x2 = fmaf(c, x0 + x0D, x2);
        } else if constexpr (KIND == kSplit) {
            x3 = fmaf(c * c, x0DR, fmaf(c, x1D, fmaf(c, x2R, x3)));
            x1 = fmaf(c, x0R, x1);
            x2 = fmaf(c, x0D, x2);
        } else if constexpr (KIND == kIntFwd) {
            // T^H then T^V; x1 one row down after T^H is recomputed.
            const V x1h = x1 - ((x0 + x0R) >> 1);
            const V x1hD = x1D - ((x0D + x0DR) >> 1);
            const V x3h = x3 - ((x2 + x2R) >> 1);
            x2 = x2 - ((x0 + x0D) >> 1);
            x3 = x3h - ((x1h + x1hD) >> 1);
            x1 = x1h;
        } else if constexpr (KIND == kIntInv) {
            // undo T^V, then T^H; x2 one column right before T^V is recomputed.
            const V x2v = x2 + ((x0 + x0D) >> 1);
            const V x3h = x3 + ((x1 + x1D) >> 1);
            const V x2Rv = x2R + ((x0R + x0DR) >> 1);
            x1 = x1 + ((x0 + x0R) >> 1);
            x3 = x3h + ((x2v + x2Rv) >> 1);
            x2 = x2v;
        }
    }
}

// ---- update-shaped block update (reads left / up / up-left) ----------------
// Operands: own x0..x3; left: x1l, x3l; up: x2u, x3u; diagonal x3ul.
template <int KIND, bool EDGE, typename V>
__device__ __forceinline__ void minus_block(V& x0, V& x1, V& x2, V& x3,
                                            V x1l, V x3l, V x2u, V x3u, V x3ul,
                                            int gc, int gr, const Geo& g, float c) {
    if constexpr (KIND == kAdj) {
        // transpose of a predict-shaped step: even[j] += c (a_j o[j] + b_j o[j-1])
        // with a_j = [j < no] + [j == no-1 && ne == no], b_j = [j >= 1]
        float ac = 1.f, bc = 1.f, ar = 1.f, br = 1.f;
        if constexpr (EDGE) {
            ac = (float)((gc < g.nOc) + (gc == g.nOc - 1 && g.nEc == g.nOc));
            bc = (gc >= 1) ? 1.f : 0.f;
            ar = (float)((gr < g.nOr) + (gr == g.nOr - 1 && g.nEr == g.nOr));
            br = (gr >= 1) ? 1.f : 0.f;
        }
        const float cc = c * c;
        const V h3 = fmaf(bc, x3l, ac * x3);
        const V h3u = fmaf(bc, x3ul, ac * x3u);
        x0 = fmaf(cc, fmaf(br, h3u, ar * h3),
                  fmaf(c, fmaf(br, x2u, ar * x2), fmaf(c, fmaf(bc, x1l, ac * x1), x0)));
        x1 = fmaf(c, fmaf(br, x3u, ar * x3), x1);
        x2 = fmaf(c, h3, x2);
    } else {
        // Symmetric extension in the polyphase domain: a neighbour index -1
        // reads index 0 and an index past the end of a component reads its
        // last sample.  Columns of x1/x3 end at nOc, rows of x2/x3 at nOr.
        const bool cO = EDGE ? (gc < g.nOc) : true;
        const bool cL = EDGE ? (gc > 0) : true;
        const bool rO = EDGE ? (gr < g.nOr) : true;
        const bool rU = EDGE ? (gr > 0) : true;
        const V x1o = cO ? x1 : x1l;          // x1 at (n, m)   clamped
        const V x1lc = cL ? x1l : x1;         // x1 at (n, m-1) clamped
        const V x3o = cO ? x3 : x3l;          // x3 at (n, m)   column-clamped
        const V x3lc = cL ? x3l : x3;         // x3 at (n, m-1)
        const V x3uo = cO ? x3u : x3ul;       // x3 at (n-1, m)
        const V x3ulc = cL ? x3ul : x3u;      // x3 at (n-1, m-1)
        const V X3oo = rO ? x3o : x3uo;       // ... and row-clamped
        const V X3ol = rO ? x3lc : x3ulc;
        const V X3uo = rU ? x3uo : x3o;
        const V X3ul = rU ? x3ulc : x3lc;
        const V x2o = rO ? x2 : x2u;          // x2 at (n, m)   clamped
        const V x2uc = rU ? x2u : x2;         // x2 at (n-1, m) clamped
        if constexpr (KIND == kFloat) {
            const float cc = c * c;
            const V s3 = (X3oo + X3ol) + (X3uo + X3ul);
            x0 = fmaf(cc, s3, fmaf(c, x2uc + x2o, fmaf(c, x1lc + x1o, x0)));
            x1 = fmaf(c, X3oo + X3uo, x1);
            x2 = fmaf(c, X3oo + X3ol, x2);
        } else if constexpr (KIND == kSplit) {
            x0 = fmaf(c * c, X3ul, fmaf(c, x2uc, fmaf(c, x1lc, x0)));
            x1 = fmaf(c, X3uo, x1);
            x2 = fmaf(c, X3ol, x2);
        } else if constexpr (KIND == kIntFwd) {
            // S^H then S^V; x2 after S^H in the row above is recomputed.
            const V x2h_own = x2 + ((x3o + x3lc + 2) >> 2);
            const V x2h_up = x2u + ((x3uo + x3ulc + 2) >> 2);
            const V x2ho = rO ? x2h_own : x2h_up;
            const V x2hu = rU ? x2h_up : x2h_own;
            x0 = x0 + ((x1lc + x1o + 2) >> 2) + ((x2ho + x2hu + 2) >> 2);
            x1 = x1 + ((X3oo + X3uo + 2) >> 2);
            x2 = x2h_own;
        } else if constexpr (KIND == kIntInv) {
            // undo S^V, then S^H; x1 before S^V one column left is recomputed.
            const V x0v = x0 - ((x2o + x2uc + 2) >> 2);
            const V x1v_own = x1 - ((X3oo + X3uo + 2) >> 2);
            const V x1v_left = x1l - ((X3ol + X3ul + 2) >> 2);
            const V x1vo = cO ? x1v_own : x1v_left;
            const V x1vl = cL ? x1v_left : x1v_own;
            x0 = x0v - ((x1vl + x1vo + 2) >> 2);
            x2 = x2 - ((X3oo + X3ol + 2) >> 2);
            x1 = x1v_own;
        }
    }
}

// ---------------------------------------------------------------------------
// whole-tile steps.  a[r][0..3] = x0..x3 of the L block of register row r,
// a[r][4..7] = x0..x3 of the R block.
// ---------------------------------------------------------------------------
template <typename V> using Row8 = V[8];

template <int K, typename V>
__device__ __forceinline__ void publish_top(V (&a)[K][8], Vec4<V> (*buf)[kLanes], int lane, int wv) {
    buf[wv][lane] = Vec4<V>{a[0][0], a[0][1], a[0][4], a[0][5]};
}
template <int K, typename V>
__device__ __forceinline__ void publish_bottom(V (&a)[K][8], Vec4<V> (*buf)[kLanes], int lane, int wv) {
    buf[wv][lane] = Vec4<V>{a[K - 1][2], a[K - 1][3], a[K - 1][6], a[K - 1][7]};
}

// Predict-shaped step over the tile: every block reads x0/x1/x2 of its right,
// lower and lower-right neighbours as they were before the step.  Rows are
// visited top to bottom so row r+1 is still unmodified when row r reads it.
template <int KIND, bool EDGE, int NW, int K, typename V>
__device__ __forceinline__ void plus_step(V (&a)[K][8], Vec4<V> (*buf)[kLanes], int lane, int wv,
                                          const Geo& g, float c) {
    V rrow = from_right(a[0][0]);                 // right lane's L.x0, row r
#pragma unroll
    for (int r = 0; r < K; ++r) {
        V dL0, dL1, dR0, dR1, dRR;
        if (r + 1 < K) {
            dL0 = a[r + 1][0]; dL1 = a[r + 1][1]; dR0 = a[r + 1][4]; dR1 = a[r + 1][5];
            dRR = from_right(a[r + 1][0]);
        } else if (wv + 1 < NW) {
            const Vec4<V> q = buf[wv + 1][lane];
            dL0 = q.a; dL1 = q.b; dR0 = q.c; dR1 = q.d;
            dRR = buf[wv + 1][lane < kLanes - 1 ? lane + 1 : lane].a;
        } else {                                  // below the tile: halo, any finite value
            dL0 = a[r][0]; dL1 = a[r][1]; dR0 = a[r][4]; dR1 = a[r][5]; dRR = rrow;
        }
        const V rR2 = from_right(a[r][2]);        // right lane's L.x2 before the step
        const int gr = g.gr0 + r;
        plus_block<KIND, EDGE>(a[r][0], a[r][1], a[r][2], a[r][3],
                               a[r][4], a[r][6], dL0, dL1, dR0, g.gcL, gr, g, c);
        plus_block<KIND, EDGE>(a[r][4], a[r][5], a[r][6], a[r][7],
                               rrow, rR2, dR0, dR1, dRR, g.gcL + 1, gr, g, c);
        rrow = dRR;
    }
}

// Update-shaped step: every block reads x1/x2/x3 of its left, upper and
// upper-left neighbours as they were before the step.  Rows are visited bottom
// to top; within a row the R block goes first because it reads the L block.
template <int KIND, bool EDGE, int NW, int K, typename V>
__device__ __forceinline__ void minus_step(V (&a)[K][8], Vec4<V> (*buf)[kLanes], int lane, int wv,
                                           const Geo& g, float c) {
    V lrow = from_left(a[K - 1][7]);              // left lane's R.x3, row r
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
        V uL2, uL3, uR2, uR3, uLL3;
        if (r > 0) {
            uL2 = a[r - 1][2]; uL3 = a[r - 1][3]; uR2 = a[r - 1][6]; uR3 = a[r - 1][7];
            uLL3 = from_left(a[r - 1][7]);
        } else if (wv > 0) {
            const Vec4<V> q = buf[wv - 1][lane];
            uL2 = q.a; uL3 = q.b; uR2 = q.c; uR3 = q.d;
            uLL3 = buf[wv - 1][lane > 0 ? lane - 1 : 0].d;
        } else {                                  // above the tile: halo
            uL2 = a[r][2]; uL3 = a[r][3]; uR2 = a[r][6]; uR3 = a[r][7]; uLL3 = lrow;
        }
        const V lL1 = from_left(a[r][5]);         // left lane's R.x1 before the step
        const int gr = g.gr0 + r;
        minus_block<KIND, EDGE>(a[r][4], a[r][5], a[r][6], a[r][7],
                                a[r][1], a[r][3], uR2, uR3, uL3, g.gcL + 1, gr, g, c);
        minus_block<KIND, EDGE>(a[r][0], a[r][1], a[r][2], a[r][3],
                                lL1, lrow, uL2, uL3, uLL3, g.gcL, gr, g, c);
        lrow = uLL3;
    }
}

// Constant parts of the split (no neighbour access): separable lifting with
// P0 = c (horizontal, then vertical) and with U0 = c.
template <int K, typename V>
__device__ __forceinline__ void local_predict(V (&a)[K][8], float c) {
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int b = 0; b < 8; b += 4) {
            a[r][b + 1] = fmaf(c, a[r][b + 0], a[r][b + 1]);
            a[r][b + 3] = fmaf(c, a[r][b + 2], a[r][b + 3]);
            a[r][b + 2] = fmaf(c, a[r][b + 0], a[r][b + 2]);
            a[r][b + 3] = fmaf(c, a[r][b + 1], a[r][b + 3]);
        }
}
template <int K, typename V>
__device__ __forceinline__ void local_update(V (&a)[K][8], float c) {
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int b = 0; b < 8; b += 4) {
            a[r][b + 0] = fmaf(c, a[r][b + 1], a[r][b + 0]);
            a[r][b + 2] = fmaf(c, a[r][b + 3], a[r][b + 2]);
            a[r][b + 0] = fmaf(c, a[r][b + 2], a[r][b + 0]);
            a[r][b + 1] = fmaf(c, a[r][b + 3], a[r][b + 1]);
        }
}
template <int K, typename V>
__device__ __forceinline__ void scale(V (&a)[K][8], float s0, float s3) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
        a[r][0] *= s0; a[r][4] *= s0;
        a[r][3] *= s3; a[r][7] *= s3;
    }
}

// The step program of one scale.  Each "sync" is the single barrier of one
// fused step; the LDS edge row it guards is published just before it.
template <int DIR, int WAV, bool EDGE, bool SPLIT, int NW, int K, typename V>
__device__ __forceinline__ void run(V (&a)[K][8], Vec4<V> (*bT)[kLanes], Vec4<V> (*bS)[kLanes],
                                    int lane, int wv, const Geo& g) {
#define DWT2_PLUS(KIND_, c_) publish_top(a, bT, lane, wv); __syncthreads(); \
    plus_step<KIND_, EDGE, NW>(a, bT, lane, wv, g, (c_));
#define DWT2_MINUS(KIND_, c_) publish_bottom(a, bS, lane, wv); __syncthreads(); \
    minus_step<KIND_, EDGE, NW>(a, bS, lane, wv, g, (c_));
    if constexpr (WAV == kCdf53) {
        if constexpr (DIR == kForward) {
            DWT2_PLUS(kIntFwd, 0.f)
            DWT2_MINUS(kIntFwd, 0.f)
        } else {
            DWT2_MINUS(kIntInv, 0.f)
            DWT2_PLUS(kIntInv, 0.f)
        }
    } else if constexpr (DIR == kForward) {
        if constexpr (SPLIT) {
            local_predict(a, kAlpha);
            DWT2_PLUS(kSplit, kAlpha) local_update(a, kBeta);
            DWT2_MINUS(kSplit, kBeta) local_predict(a, kGamma);
            DWT2_PLUS(kSplit, kGamma) local_update(a, kDelta);
            DWT2_MINUS(kSplit, kDelta)
        } else {
            DWT2_PLUS(kFloat, kAlpha)
            DWT2_MINUS(kFloat, kBeta)
            DWT2_PLUS(kFloat, kGamma)
            DWT2_MINUS(kFloat, kDelta)
        }
        scale(a, kZeta2, kZetaM2);
    } else if constexpr (DIR == kInverse) {
        scale(a, kZetaM2, kZeta2);
        if constexpr (SPLIT) {
            DWT2_MINUS(kSplit, -kDelta) local_update(a, -kDelta);
            DWT2_PLUS(kSplit, -kGamma) local_predict(a, -kGamma);
            DWT2_MINUS(kSplit, -kBeta) local_update(a, -kBeta);
            DWT2_PLUS(kSplit, -kAlpha) local_predict(a, -kAlpha);
        } else {
            DWT2_MINUS(kFloat, -kDelta)
            DWT2_PLUS(kFloat, -kGamma)
            DWT2_MINUS(kFloat, -kBeta)
            DWT2_PLUS(kFloat, -kAlpha)
        }
    } else {
        // W^T = T_1^T S_1^T T_2^T S_2^T Z: transposed steps in reverse order;
        // the transpose of an update is predict-shaped and vice versa.
        scale(a, kZeta2, kZetaM2);
        DWT2_PLUS(kAdj, kDelta)
        DWT2_MINUS(kAdj, kGamma)
        DWT2_PLUS(kAdj, kBeta)
        DWT2_MINUS(kAdj, kAlpha)
    }
#undef DWT2_PLUS
#undef DWT2_MINUS
}

// ---------------------------------------------------------------------------
// global memory access
// ---------------------------------------------------------------------------
// Four consecutive samples of one image row starting at column c (a multiple
// of 4); samples outside [0, w) or rows outside [0, h) read as 0.
template <typename T, bool EDGE>
__device__ __forceinline__ void load4(const T* base, int64_t pitch, int row, int c, int h, int w,
                                      bool vec, typename St<T>::V& v0, typename St<T>::V& v1,
                                      typename St<T>::V& v2, typename St<T>::V& v3) {
    using V = typename St<T>::V;
    v0 = v1 = v2 = v3 = V(0);
    if (EDGE && (row < 0 || row >= h || c < 0 || c >= w)) return;
    const T* p = base + (int64_t)row * pitch + c;
    if (vec && (!EDGE || c + 3 < w)) {
        const Pack4<T> q = *reinterpret_cast<const Pack4<T>*>(p);
        v0 = St<T>::load(q.v[0]); v1 = St<T>::load(q.v[1]);
        v2 = St<T>::load(q.v[2]); v3 = St<T>::load(q.v[3]);
    } else {
        v0 = St<T>::load(p[0]);
        if (!EDGE || c + 1 < w) v1 = St<T>::load(p[1]);
        if (!EDGE || c + 2 < w) v2 = St<T>::load(p[2]);
        if (!EDGE || c + 3 < w) v3 = St<T>::load(p[3]);
    }
}

template <typename T, bool EDGE>
__device__ __forceinline__ void store4(T* base, int64_t pitch, int row, int c, int h, int w, bool vec,
                                       typename St<T>::V v0, typename St<T>::V v1,
                                       typename St<T>::V v2, typename St<T>::V v3) {
    if (EDGE && (row >= h || c >= w)) return;
    T* p = base + (int64_t)row * pitch + c;
    if (vec && (!EDGE || c + 3 < w)) {
        Pack4<T> q;
        q.v[0] = St<T>::store(v0); q.v[1] = St<T>::store(v1);
        q.v[2] = St<T>::store(v2); q.v[3] = St<T>::store(v3);
        *reinterpret_cast<Pack4<T>*>(p) = q;
    } else {
        p[0] = St<T>::store(v0);
        if (!EDGE || c + 1 < w) p[1] = St<T>::store(v1);
        if (!EDGE || c + 2 < w) p[2] = St<T>::store(v2);
        if (!EDGE || c + 3 < w) p[3] = St<T>::store(v3);
    }
}

// Two consecutive samples (blocks gc, gc+1; gc even) of one subband row with
// `ncols` columns.
template <typename T, bool EDGE>
__device__ __forceinline__ void load2(const T* rowp, int gc, int ncols, bool row_ok, bool vec,
                                      typename St<T>::V& v0, typename St<T>::V& v1) {
    using V = typename St<T>::V;
    v0 = v1 = V(0);
    if (EDGE && (!row_ok || gc < 0 || gc >= ncols)) return;
    const T* p = rowp + gc;
    if (vec && (!EDGE || gc + 1 < ncols)) {
        const Pack2<T> q = *reinterpret_cast<const Pack2<T>*>(p);
        v0 = St<T>::load(q.v[0]); v1 = St<T>::load(q.v[1]);
    } else {
        v0 = St<T>::load(p[0]);
        if (!EDGE || gc + 1 < ncols) v1 = St<T>::load(p[1]);
    }
}

template <typename T, bool EDGE>
__device__ __forceinline__ void store2(T* rowp, int gc, int ncols, bool vec,
                                       typename St<T>::V v0, typename St<T>::V v1) {
    if (EDGE && gc >= ncols) return;
    T* p = rowp + gc;
    if (vec && (!EDGE || gc + 1 < ncols)) {
        Pack2<T> q;
        q.v[0] = St<T>::store(v0); q.v[1] = St<T>::store(v1);
        *reinterpret_cast<Pack2<T>*>(p) = q;
    } else {
        p[0] = St<T>::store(v0);
        if (!EDGE || gc + 1 < ncols) p[1] = St<T>::store(v1);
    }
}

// Load the tile (halo included) into registers.
template <int DIR, typename T, bool EDGE, int K>
__device__ __forceinline__ void load_tile(typename St<T>::V (&a)[K][8], const LevelParams& P, const Geo& g) {
    const bool vec = P.vec != 0;
    if constexpr (DIR == kForward) {
        const T* in = static_cast<const T*>(P.in);
        const int c = 2 * g.gcL;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int row = 2 * (g.gr0 + r);
            load4<T, EDGE>(in, P.in_pitch, row, c, P.h, P.w, vec, a[r][0], a[r][1], a[r][4], a[r][5]);
            load4<T, EDGE>(in, P.in_pitch, row + 1, c, P.h, P.w, vec, a[r][2], a[r][3], a[r][6], a[r][7]);
        }
    } else {
        const T* ll = static_cast<const T*>(P.in_ll);
        const T* det = static_cast<const T*>(P.in);
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int gr = g.gr0 + r;
            const bool rE = gr >= 0 && gr < g.nEr;
            const bool rO = gr >= 0 && gr < g.nOr;
            const int64_t gre = rE ? gr : 0, gro = rO ? gr : 0;
            load2<T, EDGE>(ll + gre * P.in_ll_pitch, g.gcL, g.nEc, rE, vec, a[r][0], a[r][4]);
            load2<T, EDGE>(det + gre * P.in_pitch + g.nEc, g.gcL, g.nOc, rE, vec, a[r][1], a[r][5]);
            load2<T, EDGE>(det + (g.nEr + gro) * P.in_pitch, g.gcL, g.nEc, rO, vec, a[r][2], a[r][6]);
            load2<T, EDGE>(det + (g.nEr + gro) * P.in_pitch + g.nEc, g.gcL, g.nOc, rO, vec, a[r][3], a[r][7]);
        }
    }
}

// Store the core of the tile (halo lanes and rows dropped).
template <int DIR, typename T, bool EDGE, int NW, int K>
__device__ __forceinline__ void store_tile(typename St<T>::V (&a)[K][8], const LevelParams& P,
                                           const Geo& g, int lane, int wv) {
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    if (lane < kHalo / 2 || lane >= kLanes - kHalo / 2) return;
    const bool vec = P.vec != 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int tr = wv * K + r;                // row within the tile
        if (tr < kHalo || tr >= kHalo + kCoreBY) continue;
        const int gr = g.gr0 + r;
        if (EDGE && gr >= g.nEr) continue;
        if constexpr (DIR == kForward) {
            T* ll = static_cast<T*>(P.out_ll);
            T* det = static_cast<T*>(P.out);
            store2<T, EDGE>(ll + (int64_t)gr * P.out_ll_pitch, g.gcL, g.nEc, vec, a[r][0], a[r][4]);
            store2<T, EDGE>(det + (int64_t)gr * P.out_pitch + g.nEc, g.gcL, g.nOc, vec, a[r][1], a[r][5]);
            if (!EDGE || gr < g.nOr) {
                store2<T, EDGE>(det + (int64_t)(g.nEr + gr) * P.out_pitch, g.gcL, g.nEc, vec, a[r][2], a[r][6]);
                store2<T, EDGE>(det + (int64_t)(g.nEr + gr) * P.out_pitch + g.nEc, g.gcL, g.nOc, vec,
                                a[r][3], a[r][7]);
            }
        } else {
            T* img = static_cast<T*>(P.out);
            const int c = 2 * g.gcL;
            store4<T, EDGE>(img, P.out_pitch, 2 * gr, c, P.h, P.w, vec, a[r][0], a[r][1], a[r][4], a[r][5]);
            store4<T, EDGE>(img, P.out_pitch, 2 * gr + 1, c, P.h, P.w, vec, a[r][2], a[r][3], a[r][6], a[r][7]);
        }
    }
}

template <int DIR, int WAV, typename T, bool SPLIT, int NW, int K>
__global__ void __launch_bounds__(NW * kLanes) level_kernel(LevelParams P) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    __shared__ Vec4<V> bufT[NW][kLanes];
    __shared__ Vec4<V> bufS[NW][kLanes];
    const int lane = threadIdx.x & (kLanes - 1);
    // the wave index is uniform: keep it (and every row address) in SGPRs
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);

    // Work-groups are dealt round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles (row-major) so neighbouring halos share its L2.
    const int nt = P.tiles_x * P.tiles_y;
    const int per = (nt + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (t >= nt) return;                          // uniform over the work-group
    const int ty = t / P.tiles_x;
    const int tx = t - ty * P.tiles_x;

    Geo g;
    g.nEr = (P.h + 1) >> 1; g.nOr = P.h >> 1;
    g.nEc = (P.w + 1) >> 1; g.nOc = P.w >> 1;
    const int cb0 = tx * kCoreBX, rb0 = ty * kCoreBY;
    g.gcL = cb0 - kHalo + 2 * lane;
    g.gr0 = rb0 - kHalo + wv * K;
    // Interior tile: every loaded block has all four components and no
    // neighbour index of the core's dependency cone needs clamping.
    const bool interior = rb0 - kHalo >= 0 && cb0 - kHalo >= 0 &&
                          rb0 + kCoreBY + kHalo <= g.nOr && cb0 + kCoreBX + kHalo <= g.nOc;
    V a[K][8];
    if (interior) {
        load_tile<DIR, T, false>(a, P, g);
        run<DIR, WAV, false, SPLIT, NW>(a, bufT, bufS, lane, wv, g);
        store_tile<DIR, T, false, NW>(a, P, g, lane, wv);
    } else {
        load_tile<DIR, T, true>(a, P, g);
        run<DIR, WAV, true, false, NW>(a, bufT, bufS, lane, wv, g);
        store_tile<DIR, T, true, NW>(a, P, g, lane, wv);
    }
}

template <int DIR, int WAV, typename T, bool SPLIT, int NW, int K>
hipError_t launch_shape(const LevelParams& p, hipStream_t s) {
    const int nt = p.tiles_x * p.tiles_y;
    const int grid = ((nt + 7) >> 3) * 8;
    hipLaunchKernelGGL((level_kernel<DIR, WAV, T, SPLIT, NW, K>), dim3(grid), dim3(NW * kLanes), 0, s, p);
    return hipGetLastError();
}

template <int DIR, int WAV, typename T, bool SPLIT>
hipError_t launch(int shape, const LevelParams& p, hipStream_t s) {
    static_assert(kNumTileShapes == 6, "dispatch table below lists every tile shape");
    switch (shape) {
        case 0: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[0].waves, kTileShapes[0].rows>(p, s);
        case 1: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[1].waves, kTileShapes[1].rows>(p, s);
        case 2: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[2].waves, kTileShapes[2].rows>(p, s);
        case 3: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[3].waves, kTileShapes[3].rows>(p, s);
        case 4: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[4].waves, kTileShapes[4].rows>(p, s);
        case 5: return launch_shape<DIR, WAV, T, SPLIT, kTileShapes[5].waves, kTileShapes[5].rows>(p, s);
    }
    return hipErrorInvalidValue;
}

template <int DIR, typename T>
hipError_t launch_float(bool split, int shape, const LevelParams& p, hipStream_t s) {
    if constexpr (DIR == kAdjoint) {
        return launch<DIR, kCdf97, T, false>(shape, p, s);
    } else {
        return split ? launch<DIR, kCdf97, T, true>(shape, p, s) : launch<DIR, kCdf97, T, false>(shape, p, s);
    }
}

template <int DIR>
hipError_t launch_dir(Wavelet wav, Dtype dt, bool split, int shape, const LevelParams& p, hipStream_t s) {
    if (wav == kCdf53) {
        if constexpr (DIR == kAdjoint) return hipErrorInvalidValue;
        else return launch<DIR, kCdf53, int32_t, false>(shape, p, s);
    }
    switch (dt) {
        case kF32: return launch_float<DIR, float>(split, shape, p, s);
        case kBF16: return launch_float<DIR, __hip_bfloat16>(split, shape, p, s);
        case kF16: return launch_float<DIR, __half>(split, shape, p, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_level(Direction dir, Wavelet wav, Dtype dt, bool split, int shape,
                        const LevelParams& p, hipStream_t stream) {
    if (p.tiles_x <= 0 || p.tiles_y <= 0) return hipSuccess;
    switch (dir) {
        case kForward: return launch_dir<kForward>(wav, dt, split, shape, p, stream);
        case kInverse: return launch_dir<kInverse>(wav, dt, split, shape, p, stream);
        case kAdjoint: return launch_dir<kAdjoint>(wav, dt, split, shape, p, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace dwt2
