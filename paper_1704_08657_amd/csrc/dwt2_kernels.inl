// Device code shared by the per-direction translation units (dwt2_fwd.hip,
// dwt2_inv.hip, dwt2_adj.hip); included, not compiled on its own.
#pragma once
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
//   * one work-group = NW wave64s = one tile of (64 * BPL) x (NW * K) blocks
//     (e.g. 256 x 32 pixels for BPL = 2, NW = K = 4) with a 2-block halo
//     recomputed on every side;
//   * each lane owns BPL horizontally adjacent blocks (2 or 4) for K
//     consecutive block rows, all in VGPRs, plus a halo pair used by the
//     first and last lane only;
//   * a step reads neighbours at +1 (predict-shaped: right / down) or at -1
//     (update-shaped: left / up).  Horizontal neighbours come from the
//     adjacent lane through DPP wave shifts, vertical ones from the lane's own
//     registers, except at the boundary between two waves, where the edge row
//     is published to LDS before the step's single s_barrier (two LDS buffers,
//     one for each step shape, so one barrier per step suffices);
//   * loads are 4-pixel vectors per image row, stores are BPL-sample vectors
//     per subband row, both coalesced across the wave;
//   * tiles touching the image border load the whole-point symmetric
//     extension of the image and then run the same unclamped steps (each
//     step keeps the extension symmetric); the adjoint's border tiles apply
//     the transposed border weights instead; interior tiles take a
//     branch-free vector path;
//   * the step program is chosen at compile time: the fused steps, the fused
//     steps with the split, the separable steps (the comparison scheme) or
//     the fused steps evaluated as their two 1-D factors;
//   * the tile index is remapped so that each XCD (work-groups are dealt
//     round-robin over the 8 XCDs) takes whole rows of tiles, so the halo
//     re-reads of neighbouring tiles hit that XCD's L2.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dwt2_internal.h"

namespace dwt2 {
namespace kern {

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
// Real-valued CDF 5/3: one pair, predict -1/2, update 1/4; the same
// normalisation gives zeta = sqrt(2): LL * 2, HH * 1/2 (exact in FP32).
constexpr float kP53 = -0.5f;
constexpr float kU53 = 0.25f;
constexpr float kZeta53Sq = 2.0f;
constexpr float kZeta53SqInv = 0.5f;


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
    // The conversion is one explicit instruction on the finished FP32 value,
    // so the compiler cannot merge it with the multiply-add that produced
    // the value (a mixed-precision FMA rounds once, straight to FP16, and in
    // rare cases differs by one FP16 unit): every kernel rounds the same way.
    __device__ static __half store(V v) {
        unsigned r;
        asm("v_cvt_f16_f32 %0, %1" : "=v"(r) : "v"(v));
        return __ushort_as_half((unsigned short)r);
    }
};
template <> struct St<int32_t> {
    using V = int;
    __device__ static V load(int32_t v) { return v; }
    __device__ static int32_t store(V v) { return v; }
};

template <typename T> struct alignas(8 * sizeof(T)) Pack8 { T v[8]; };
template <typename T> struct alignas(4 * sizeof(T)) Pack4 { T v[4]; };
template <typename T> struct alignas(2 * sizeof(T)) Pack2 { T v[2]; };
static_assert(sizeof(Pack4<float>) == 16 && sizeof(Pack2<__half>) == 4, "packed vector layout");

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
// Same shifts, but the lane without a source lane (63 for from_right, 0 for
// from_left) keeps `old` instead (bound_ctrl off): one instruction replaces a
// shift plus a lane select.
__device__ __forceinline__ float from_right_or(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_left_or(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ int from_right_or(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ int from_left_or(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}

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
    kIntInv = 5,     // reversible 5/3 inverse
    // separable steps (the comparison scheme): one axis per step
    kSepH = 6,       // float horizontal step (coefficient sign as given)
    kSepV = 7,       // float vertical step
    kSepHInt = 8,    // reversible 5/3 forward, horizontal
    kSepVInt = 9,    // reversible 5/3 forward, vertical
    kSepHIntInv = 10,  // reversible 5/3 inverse, horizontal
    kSepVIntInv = 11   // reversible 5/3 inverse, vertical
};

template <typename V> struct alignas(4 * sizeof(V)) Vec4 { V a, b, c, d; };
template <typename V> struct alignas(2 * sizeof(V)) Vec2 { V a, b; };

// ---- predict-shaped block update (reads right / down / down-right) --------
// Operands: own x0..x3; right: x0R, x2R; down: x0D, x1D; diagonal x0DR.
template <int KIND, bool EX, bool EY, typename V>
__device__ __forceinline__ void plus_block(V& x0, V& x1, V& x2, V& x3,
                                           V x0R, V x2R, V x0D, V x1D, V x0DR,
                                           int gc, int gr, const Geo& g, float c) {
    if constexpr (KIND == kAdj) {
        // transpose of an update-shaped step: odd[k] += c (al_k e[k] + be_k e[k+1])
        // with al_k = 1 + [k == 0], be_k = [k+1 < ne] + [k+1 == no && ne > no]
        float alc = 1.f, bec = 1.f, alr = 1.f, ber = 1.f;
        if constexpr (EX) {
            alc = (gc == 0) ? 2.f : 1.f;
            bec = (float)((gc + 1 < g.nEc) + (gc + 1 == g.nOc && g.nEc > g.nOc));
        }
        if constexpr (EY) {
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
        if constexpr (EX || EY) {
            const bool cR = EX ? (gc + 1 < g.nEc) : true;
            const bool rD = EY ? (gr + 1 < g.nEr) : true;
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
        } else if constexpr (KIND == kSepH) {        // T^H: odd columns from the even ones
            x1 = fmaf(c, x0 + x0R, x1);
            x3 = fmaf(c, x2 + x2R, x3);
        } else if constexpr (KIND == kSepV) {        // T^V: odd rows from the even ones
            x2 = fmaf(c, x0 + x0D, x2);
            x3 = fmaf(c, x1 + x1D, x3);
        } else if constexpr (KIND == kSepHInt) {
            x1 = x1 - ((x0 + x0R) >> 1);
            x3 = x3 - ((x2 + x2R) >> 1);
        } else if constexpr (KIND == kSepVInt) {
            x2 = x2 - ((x0 + x0D) >> 1);
            x3 = x3 - ((x1 + x1D) >> 1);
        } else if constexpr (KIND == kSepHIntInv) {
            x1 = x1 + ((x0 + x0R) >> 1);
            x3 = x3 + ((x2 + x2R) >> 1);
        } else if constexpr (KIND == kSepVIntInv) {
            x2 = x2 + ((x0 + x0D) >> 1);
            x3 = x3 + ((x1 + x1D) >> 1);
        }
    }
}

// ---- update-shaped block update (reads left / up / up-left) ----------------
// Operands: own x0..x3; left: x1l, x3l; up: x2u, x3u; diagonal x3ul.
template <int KIND, bool EX, bool EY, typename V>
__device__ __forceinline__ void minus_block(V& x0, V& x1, V& x2, V& x3,
                                            V x1l, V x3l, V x2u, V x3u, V x3ul,
                                            int gc, int gr, const Geo& g, float c) {
    if constexpr (KIND == kAdj) {
        // transpose of a predict-shaped step: even[j] += c (a_j o[j] + b_j o[j-1])
        // with a_j = [j < no] + [j == no-1 && ne == no], b_j = [j >= 1]
        float ac = 1.f, bc = 1.f, ar = 1.f, br = 1.f;
        if constexpr (EX) {
            ac = (float)((gc < g.nOc) + (gc == g.nOc - 1 && g.nEc == g.nOc));
            bc = (gc >= 1) ? 1.f : 0.f;
        }
        if constexpr (EY) {
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
        const bool cO = EX ? (gc < g.nOc) : true;
        const bool cL = EX ? (gc > 0) : true;
        const bool rO = EY ? (gr < g.nOr) : true;
        const bool rU = EY ? (gr > 0) : true;
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
        } else if constexpr (KIND == kSepH) {        // S^H: even columns from the odd ones
            x0 = fmaf(c, x1lc + x1o, x0);
            x2 = fmaf(c, X3oo + X3ol, x2);
        } else if constexpr (KIND == kSepV) {        // S^V: even rows from the odd ones
            x0 = fmaf(c, x2uc + x2o, x0);
            x1 = fmaf(c, X3oo + X3uo, x1);
        } else if constexpr (KIND == kSepHInt) {
            x0 = x0 + ((x1lc + x1o + 2) >> 2);
            x2 = x2 + ((X3oo + X3ol + 2) >> 2);
        } else if constexpr (KIND == kSepVInt) {
            x0 = x0 + ((x2uc + x2o + 2) >> 2);
            x1 = x1 + ((X3oo + X3uo + 2) >> 2);
        } else if constexpr (KIND == kSepHIntInv) {
            x0 = x0 - ((x1lc + x1o + 2) >> 2);
            x2 = x2 - ((X3oo + X3ol + 2) >> 2);
        } else if constexpr (KIND == kSepVIntInv) {
            x0 = x0 - ((x2uc + x2o + 2) >> 2);
            x1 = x1 - ((X3oo + X3uo + 2) >> 2);
        }
    }
}

// ---------------------------------------------------------------------------
// Tile kernel.  A lane holds BPL horizontally adjacent blocks (tile columns
// BPL*lane .. BPL*lane + BPL - 1) for each of its K block rows, so a wave
// covers the tile's 64 * BPL output columns, aligned to whole subband rows
// of 64 * BPL samples: every store covers whole cache lines.
// a[r][4 b + k] = component x_k of core block b of row r.
//
// The horizontal halo (two block columns on each side) is held in one more
// register pair, e[8], with its rows spread over lanes: lane q < 32 holds
// the two halo blocks of the wave's block row r = q & 15 (if r < K) on side
// q >> 4 (side 0: tile columns -2, -1; side 1: 64*BPL, 64*BPL + 1);
// e[0..3] = x0..x3 of the first block, e[4..7] of the second.  A fused step
// thus updates the halo with two block updates for the whole wave instead of
// two per row.  Vertical neighbours of halo blocks are the adjacent lanes
// (DPP row shifts); the values that cross between the halo lanes and the
// first / last lane of the core go through a small per-wave LDS area.
// ---------------------------------------------------------------------------
template <int BPL> struct Lay {
    static_assert(BPL == 2 || BPL == 4, "2 or 4 blocks per lane");
    static constexpr int BX = 4 * BPL;            // values per register row
    static constexpr int LAST = 4 * (BPL - 1);    // last block
    static constexpr int NG = BPL / 2;            // Vec4 groups of one edge row (2 values per block)
    static constexpr int CORE_BX = kLanes * BPL;  // output block columns of a tile
};

// lane i <- lane i+1 (next) or i-1 (prev) within its row of 16 lanes (0 in
// a lane without a source lane in its row).
__device__ __forceinline__ int row_next(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x101 /* row_shl:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ int row_prev(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x111 /* row_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ float row_next(float v) { return __int_as_float(row_next(__float_as_int(v))); }
__device__ __forceinline__ float row_prev(float v) { return __int_as_float(row_prev(__float_as_int(v))); }

// LDS of one work-group.  t: the top block row (x0, x1) of every wave, for
// the wave above; s: the bottom row (x2, x3), for the wave below; both
// group-major (buf[wave][group][lane], 16-byte accesses contiguous across
// the wave).  et / es: the same for the halo rows (per side: first block,
// second block).  Wave w publishes to t[w], et[w], s[w + 1], es[w + 1] and
// reads t[w + 1], et[w + 1], s[w], es[w]: the slots t[NW], s[0] (and the
// halo ones) hold zeros for the outermost waves, which only reach tile rows
// outside the core (a predict-shaped step carries values up one row, an
// update-shaped one down one row, and the tile's 2-row halo absorbs the two
// of each).  col / hal: per-wave exchange
// between the core's edge lane and the halo lanes, indexed by block row.
template <typename V, int NW, int BPL, int K> struct TileLds {
    static_assert(K % 2 == 0 && K <= 16, "K even, at most 16 rows per wave");
    Vec4<V> t[NW + 1][Lay<BPL>::NG][kLanes];
    Vec4<V> s[NW + 1][Lay<BPL>::NG][kLanes];
    Vec4<V> et[NW + 1][2];
    Vec4<V> es[NW + 1][2];
    V col[NW][2][16];
    V hal[NW][2][16];
};

// Operands of a predict-shaped step for N blocks, all taken before the step:
// right neighbour (x0R, x2R), lower (x0D, x1D), lower-right (x0DR).
template <typename V, int N> struct PlusOps { V x0R[N], x2R[N], x0D[N], x1D[N], x0DR[N]; };
// Operands of an update-shaped step: left (x1l, x3l), upper (x2u, x3u), upper-left (x3ul).
template <typename V, int N> struct MinusOps { V x1l[N], x3l[N], x2u[N], x3u[N], x3ul[N]; };

// cur: the row; dn: the row below (x0, x1 used).  The right neighbour of the
// last block is the next lane's first block: R0, R2 are that block's x0, x2
// for this row and RD0 its x0 for the row below (lane 63: the halo column
// 64*BPL instead).
template <int BPL, typename V>
__device__ __forceinline__ void gather_plus(const V (&cur)[Lay<BPL>::BX], const V (&dn)[Lay<BPL>::BX], V R0, V R2,
                                            V RD0, PlusOps<V, BPL>& o) {
    using L = Lay<BPL>;
#pragma unroll
    for (int b = 0; b + 1 < BPL; ++b) {
        o.x0R[b] = cur[4 * b + 4]; o.x2R[b] = cur[4 * b + 6];
        o.x0D[b] = dn[4 * b]; o.x1D[b] = dn[4 * b + 1]; o.x0DR[b] = dn[4 * b + 4];
    }
    constexpr int b = BPL - 1;
    o.x0R[b] = R0; o.x2R[b] = R2;
    o.x0D[b] = dn[L::LAST]; o.x1D[b] = dn[L::LAST + 1]; o.x0DR[b] = RD0;
}

// cur: the row; up: the row above (x2, x3 used).  The left neighbour of the
// first block is the previous lane's last block: L1, L3 are that block's
// x1, x3 for this row and LU3 its x3 for the row above (lane 0: the halo
// column -1 instead).
template <int BPL, typename V>
__device__ __forceinline__ void gather_minus(const V (&cur)[Lay<BPL>::BX], const V (&up)[Lay<BPL>::BX], V L1, V L3,
                                             V LU3, MinusOps<V, BPL>& o) {
    o.x1l[0] = L1; o.x3l[0] = L3;
    o.x2u[0] = up[2]; o.x3u[0] = up[3]; o.x3ul[0] = LU3;
#pragma unroll
    for (int b = 1; b < BPL; ++b) {
        o.x1l[b] = cur[4 * b - 3]; o.x3l[b] = cur[4 * b - 1];
        o.x2u[b] = up[4 * b + 2]; o.x3u[b] = up[4 * b + 3]; o.x3ul[b] = up[4 * b - 1];
    }
}

// Apply a step to blocks 0 .. N-1 of v (v[4 b + k] = x_k of block b) whose
// bit is set in MASK; gc[b]: block column, gr: block row.
template <int KIND, int MASK, bool EX, bool EY, int N, typename V>
__device__ __forceinline__ void apply_plus(V (&v)[4 * N], const PlusOps<V, N>& o, const int (&gc)[N], int gr,
                                           const Geo& g, float c) {
#pragma unroll
    for (int b = 0; b < N; ++b)
        if ((MASK >> b) & 1)
            plus_block<KIND, EX, EY>(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3], o.x0R[b], o.x2R[b],
                                     o.x0D[b], o.x1D[b], o.x0DR[b], gc[b], gr, g, c);
}
template <int KIND, int MASK, bool EX, bool EY, int N, typename V>
__device__ __forceinline__ void apply_minus(V (&v)[4 * N], const MinusOps<V, N>& o, const int (&gc)[N], int gr,
                                            const Geo& g, float c) {
#pragma unroll
    for (int b = 0; b < N; ++b)
        if ((MASK >> b) & 1)
            minus_block<KIND, EX, EY>(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3], o.x1l[b], o.x3l[b],
                                      o.x2u[b], o.x3u[b], o.x3ul[b], gc[b], gr, g, c);
}

// Edge rows of the core for the neighbouring waves: x_k0, x_k0+1 of every
// block (k0 = 0: top row for predict-shaped steps, 2: bottom row for
// update-shaped steps).
template <int BPL, typename V>
__device__ __forceinline__ void publish_row(const V (&row)[Lay<BPL>::BX], int k0, Vec4<V> (*buf)[kLanes],
                                            int lane) {
#pragma unroll
    for (int q = 0; q < Lay<BPL>::NG; ++q)
        buf[q][lane] = Vec4<V>{row[8 * q + k0], row[8 * q + k0 + 1], row[8 * q + 4 + k0], row[8 * q + 4 + k0 + 1]};
}
template <int BPL, typename V>
__device__ __forceinline__ void fetch_row(V (&row)[Lay<BPL>::BX], int k0, Vec4<V> (*buf)[kLanes], int lane) {
#pragma unroll
    for (int q = 0; q < Lay<BPL>::NG; ++q) {
        const Vec4<V> v = buf[q][lane];
        row[8 * q + k0] = v.a; row[8 * q + k0 + 1] = v.b;
        row[8 * q + 4 + k0] = v.c; row[8 * q + 4 + k0 + 1] = v.d;
    }
}

// Per-lane geometry of a tile step.
template <int BPL> struct TileGeo {
    int gc[BPL];      // block columns of the lane's core blocks
    int ge[2];        // block columns of the lane's halo blocks
    int gre;          // block row of the lane's halo row
    int re;           // halo row within the wave (lane & 15)
};

// Before the barrier of a predict-shaped step: the wave's top rows (core and
// halo) for the wave above (PV), and the exchange columns for this wave (PH):
// core column 0 (x0, x2 of every row, read by the left halo lanes) and halo
// column 64*BPL (x0, x2, read by lane 63).  A fused step needs both; a
// separable step only those of its own axis.
template <int NW, int BPL, int K, bool PH = true, bool PV = true, typename V>
__device__ __forceinline__ void publish_plus(const V (&a)[K][Lay<BPL>::BX], const V (&e)[8],
                                             TileLds<V, NW, BPL, K>& L, int lane, int wv) {
    if constexpr (PV) {
        publish_row<BPL>(a[0], 0, L.t[wv], lane);
        if (lane < 32 && (lane & 15) == 0) L.et[wv][lane >> 4] = Vec4<V>{e[0], e[1], e[4], e[5]};
    }
    if constexpr (!PH) return;
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < K; r += 2) {
            *reinterpret_cast<Vec2<V>*>(&L.col[wv][0][r]) = Vec2<V>{a[r][0], a[r + 1][0]};
            *reinterpret_cast<Vec2<V>*>(&L.col[wv][1][r]) = Vec2<V>{a[r][2], a[r + 1][2]};
        }
    }
    if (lane >= 16 && lane < 16 + K) {
        L.hal[wv][0][lane - 16] = e[0];
        L.hal[wv][1][lane - 16] = e[2];
    }
}

// Before the barrier of an update-shaped step: the bottom rows for the wave
// below, core column 64*BPL - 1 (x1, x3, read by the right halo lanes) and
// halo column -1 (x1, x3, read by lane 0).
template <int NW, int BPL, int K, bool PH = true, bool PV = true, typename V>
__device__ __forceinline__ void publish_minus(const V (&a)[K][Lay<BPL>::BX], const V (&e)[8],
                                              TileLds<V, NW, BPL, K>& L, int lane, int wv) {
    using Ly = Lay<BPL>;
    if constexpr (PV) {
        publish_row<BPL>(a[K - 1], 2, L.s[wv + 1], lane);
        if (lane < 32 && (lane & 15) == K - 1) L.es[wv + 1][lane >> 4] = Vec4<V>{e[2], e[3], e[6], e[7]};
    }
    if constexpr (!PH) return;
    if (lane == kLanes - 1) {
#pragma unroll
        for (int r = 0; r < K; r += 2) {
            *reinterpret_cast<Vec2<V>*>(&L.col[wv][0][r]) = Vec2<V>{a[r][Ly::LAST + 1], a[r + 1][Ly::LAST + 1]};
            *reinterpret_cast<Vec2<V>*>(&L.col[wv][1][r]) = Vec2<V>{a[r][Ly::LAST + 3], a[r + 1][Ly::LAST + 3]};
        }
    }
    if (lane < K) {
        L.hal[wv][0][lane] = e[5];
        L.hal[wv][1][lane] = e[7];
    }
}

// Predict-shaped step over the tile (after the barrier).  Core rows top to
// bottom, so row r+1 is still unmodified when row r reads it; the halo lanes
// read only values taken before the step.
template <int KIND, int EMASK, bool EDGE, int NW, int BPL, int K, typename V>
__device__ __forceinline__ void plus_step(V (&a)[K][Lay<BPL>::BX], V (&e)[8], TileLds<V, NW, BPL, K>& L, int lane,
                                          int wv, const Geo& g, const TileGeo<BPL>& tg, float c) {
    using Ly = Lay<BPL>;
    // halo operands first (e is still at the previous stage)
    PlusOps<V, 2> h;
    {
        const int side = (lane >> 4) & 1;
        const Vec4<V> q = L.et[wv + 1][side];
        const V n0 = q.a, n1 = q.b, n2 = q.c, n3 = q.d;
        const bool last = tg.re == K - 1;
        // the halo row below: the next lane, or the next wave's top halo row
        const V s00 = row_next(e[0]), s01 = row_next(e[1]), s10 = row_next(e[4]), s11 = row_next(e[5]);
        const V d00 = last ? n0 : s00;
        const V d01 = last ? n1 : s01;
        const V d10 = last ? n2 : s10;
        const V d11 = last ? n3 : s11;
        // right of the second halo block: core column 0 (left side; on the
        // right side the outermost halo, where any value will do)
        const V cR0 = L.col[wv][0][tg.re];
        const V cR2 = L.col[wv][1][tg.re];
        const V cDR0 = tg.re + 1 < K ? L.col[wv][0][min(tg.re + 1, 15)] : L.t[wv + 1][0][0].a;
        h.x0R[0] = e[4]; h.x2R[0] = e[6]; h.x0D[0] = d00; h.x1D[0] = d01; h.x0DR[0] = d10;
        h.x0R[1] = cR0;  h.x2R[1] = cR2;  h.x0D[1] = d10; h.x1D[1] = d11; h.x0DR[1] = cDR0;
    }
    // x0, x2 of the right neighbour of each row's last block (x0 is not
    // changed by a predict-shaped step, so row r+1's value is also row r's
    // lower-right operand)
    V dn[Ly::BX];                                 // the row below the wave
    fetch_row<BPL>(dn, 0, L.t[wv + 1], lane);
    V R0[K + 1], R2[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        R0[r] = from_right_or(L.hal[wv][0][r], a[r][0]);
        R2[r] = from_right_or(L.hal[wv][1][r], a[r][2]);
    }
    R0[K] = from_right_or(L.et[wv + 1][1].a, dn[0]);
#pragma unroll
    for (int r = 0; r < K; ++r) {
        PlusOps<V, BPL> o;
        if (r + 1 < K) gather_plus<BPL>(a[r], a[r + 1 < K ? r + 1 : r], R0[r], R2[r], R0[r + 1], o);
        else gather_plus<BPL>(a[r], dn, R0[r], R2[r], R0[r + 1], o);
        apply_plus<KIND, (1 << BPL) - 1, EDGE, EDGE>(a[r], o, tg.gc, g.gr0 + r, g, c);
    }
    apply_plus<KIND, EMASK, EDGE, EDGE>(e, h, tg.ge, tg.gre, g, c);
}

// Update-shaped step over the tile (after the barrier): core rows bottom to top.
template <int KIND, int EMASK, bool EDGE, int NW, int BPL, int K, typename V>
__device__ __forceinline__ void minus_step(V (&a)[K][Lay<BPL>::BX], V (&e)[8], TileLds<V, NW, BPL, K>& L, int lane,
                                           int wv, const Geo& g, const TileGeo<BPL>& tg, float c) {
    using Ly = Lay<BPL>;
    MinusOps<V, 2> h;
    {
        const int side = (lane >> 4) & 1;
        const Vec4<V> q = L.es[wv][side];
        const V p0 = q.a, p1 = q.b, p2 = q.c, p3 = q.d;
        // the halo row above: the previous lane, or for the wave's first row
        // the previous wave's bottom halo row
        const bool first = tg.re == 0;
        const V s02 = row_prev(e[2]), s03 = row_prev(e[3]), s12 = row_prev(e[6]), s13 = row_prev(e[7]);
        const V u02 = first ? p0 : s02;
        const V u03 = first ? p1 : s03;
        const V u12 = first ? p2 : s12;
        const V u13 = first ? p3 : s13;
        // left of the first halo block: core column 64*BPL - 1 (right side;
        // on the left side the outermost halo)
        const V cL1 = L.col[wv][0][tg.re];
        const V cL3 = L.col[wv][1][tg.re];
        const V cUL3 = tg.re > 0 ? L.col[wv][1][max(tg.re - 1, 0)] : L.s[wv][Ly::NG - 1][kLanes - 1].d;
        h.x1l[0] = cL1;  h.x3l[0] = cL3;  h.x2u[0] = u02; h.x3u[0] = u03; h.x3ul[0] = cUL3;
        h.x1l[1] = e[1]; h.x3l[1] = e[3]; h.x2u[1] = u12; h.x3u[1] = u13; h.x3ul[1] = u03;
    }
    // x1, x3 of the left neighbour of each row's first block (x3 is not
    // changed by an update-shaped step, so row r-1's value is also row r's
    // upper-left operand); index r + 1 holds row r
    V up[Ly::BX];                                 // the row above the wave
    fetch_row<BPL>(up, 2, L.s[wv], lane);
    V L1[K], L3[K + 1];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        L1[r] = from_left_or(L.hal[wv][0][r], a[r][Ly::LAST + 1]);
        L3[r + 1] = from_left_or(L.hal[wv][1][r], a[r][Ly::LAST + 3]);
    }
    L3[0] = from_left_or(L.es[wv][0].d, up[Ly::LAST + 3]);
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
        MinusOps<V, BPL> o;
        if (r > 0) gather_minus<BPL>(a[r], a[r > 0 ? r - 1 : 0], L1[r], L3[r + 1], L3[r], o);
        else gather_minus<BPL>(a[r], up, L1[r], L3[r + 1], L3[r], o);
        apply_minus<KIND, (1 << BPL) - 1, EDGE, EDGE>(a[r], o, tg.gc, g.gr0 + r, g, c);
    }
    apply_minus<KIND, EMASK, EDGE, EDGE>(e, h, tg.ge, tg.gre, g, c);
}

// Constant parts of the split (no neighbour access): separable lifting with
// P0 = c (horizontal, then vertical) and with U0 = c, for every block.
template <typename V>
__device__ __forceinline__ void local_predict_block(V* v, float c) {
    v[1] = fmaf(c, v[0], v[1]);
    v[3] = fmaf(c, v[2], v[3]);
    v[2] = fmaf(c, v[0], v[2]);
    v[3] = fmaf(c, v[1], v[3]);
}
template <typename V>
__device__ __forceinline__ void local_update_block(V* v, float c) {
    v[0] = fmaf(c, v[1], v[0]);
    v[2] = fmaf(c, v[3], v[2]);
    v[0] = fmaf(c, v[2], v[0]);
    v[1] = fmaf(c, v[3], v[1]);
}
template <int K, int BX, typename V>
__device__ __forceinline__ void local_predict(V (&a)[K][BX], V (&e)[8], float c) {
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int b = 0; b < BX; b += 4) local_predict_block(&a[r][b], c);
    local_predict_block(&e[0], c);
    local_predict_block(&e[4], c);
}
template <int K, int BX, typename V>
__device__ __forceinline__ void local_update(V (&a)[K][BX], V (&e)[8], float c) {
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int b = 0; b < BX; b += 4) local_update_block(&a[r][b], c);
    local_update_block(&e[0], c);
    local_update_block(&e[4], c);
}
template <int K, int BX, typename V>
__device__ __forceinline__ void scale(V (&a)[K][BX], V (&e)[8], float s0, float s3) {
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int b = 0; b < BX; b += 4) {
            a[r][b + 0] *= s0;
            a[r][b + 3] *= s3;
        }
    e[0] *= s0; e[3] *= s3; e[4] *= s0; e[7] *= s3;
}

// Synchronisation before the horizontal factor of a step.  The separable
// scheme takes a work-group barrier there, as the paper's separable lifting
// does.  In the factored scheme the horizontal factor reads only values of
// its own wave (DPP and the wave's own LDS exchange columns; a wave's LDS
// accesses execute in program order), so no barrier is needed: the fused
// step keeps its single barrier, before its vertical factor.
template <int SCH>
__device__ __forceinline__ void sync_horizontal() {
    if constexpr (SCH == kSchemeSeparable) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// The step program of one scale.  Each "sync" is the single barrier of one
// step; the LDS rows it guards are published just before it.  SCH selects
// the fused steps (4 barriers for CDF 9/7, 2 for 5/3), the fused steps with
// the split, the separable steps (8 and 4 barriers), or the fused steps
// evaluated as their horizontal and vertical factors (4 and 2 barriers).
template <int DIR, int WAV, bool EDGE, int SCH, int NW, int BPL, int K, typename V>
__device__ __forceinline__ void run(V (&a)[K][Lay<BPL>::BX], V (&e)[8], TileLds<V, NW, BPL, K>& L, int lane, int wv,
                                    const Geo& g, const TileGeo<BPL>& tg) {
    // the slots no wave publishes to hold zeros (the transposed border
    // weights multiply values beyond the tile by 0, which must stay finite)
    if (wv == NW - 1) {
#pragma unroll
        for (int q = 0; q < Lay<BPL>::NG; ++q) L.t[NW][q][lane] = Vec4<V>{V(0), V(0), V(0), V(0)};
        if (lane < 2) L.et[NW][lane] = Vec4<V>{V(0), V(0), V(0), V(0)};
    }
    if (wv == 0) {
#pragma unroll
        for (int q = 0; q < Lay<BPL>::NG; ++q) L.s[0][q][lane] = Vec4<V>{V(0), V(0), V(0), V(0)};
        if (lane < 2) L.es[0][lane] = Vec4<V>{V(0), V(0), V(0), V(0)};
    }
#define DWT2_PLUS(KIND_, M_, c_) publish_plus<NW, BPL, K>(a, e, L, lane, wv); __syncthreads(); \
    plus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
#define DWT2_MINUS(KIND_, M_, c_) publish_minus<NW, BPL, K>(a, e, L, lane, wv); __syncthreads(); \
    minus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
    // separable steps publish only what their axis reads: exchange columns
    // (horizontal) or edge rows (vertical)
#define DWT2_PH(KIND_, M_, c_) publish_plus<NW, BPL, K, true, false>(a, e, L, lane, wv); sync_horizontal<SCH>(); \
    plus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
#define DWT2_PV(KIND_, M_, c_) publish_plus<NW, BPL, K, false, true>(a, e, L, lane, wv); __syncthreads(); \
    plus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
#define DWT2_MH(KIND_, M_, c_) publish_minus<NW, BPL, K, true, false>(a, e, L, lane, wv); sync_horizontal<SCH>(); \
    minus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
#define DWT2_MV(KIND_, M_, c_) publish_minus<NW, BPL, K, false, true>(a, e, L, lane, wv); __syncthreads(); \
    minus_step<KIND_, M_, EDGE, NW, BPL, K>(a, e, L, lane, wv, g, tg, (c_));
    // halo masks (first halo block = 1, second = 2) per step, from the column ranges each stage
    // must cover: predict/update/predict/update -> 3, 3, 2, 0;
    // update/predict/update/predict -> 3, 3, 1, 0; predict/update -> 2, 0;
    // update/predict -> 1, 0.  Separable: a vertical step keeps the mask of
    // the horizontal step before it (forward 3,3,3,3,2,2,0,0; inverse
    // 3,3,3,3,3,1,1,0; 5/3 forward 2,2,0,0; 5/3 inverse 3,1,1,0).
    if constexpr (SCH == kSchemeSeparable || SCH == kSchemeFactored) {
        static_assert(DIR != kAdjoint, "the separable and factored schemes have no adjoint");
        if constexpr (WAV == kCdf53) {
            if constexpr (DIR == kForward) {
                DWT2_PH(kSepHInt, 2, 0.f) DWT2_PV(kSepVInt, 2, 0.f)
                DWT2_MH(kSepHInt, 0, 0.f) DWT2_MV(kSepVInt, 0, 0.f)
            } else {
                DWT2_MV(kSepVIntInv, 3, 0.f) DWT2_MH(kSepHIntInv, 1, 0.f)
                DWT2_PV(kSepVIntInv, 1, 0.f) DWT2_PH(kSepHIntInv, 0, 0.f)
            }
        } else if constexpr (WAV == kCdf53Real) {
            if constexpr (DIR == kForward) {
                DWT2_PH(kSepH, 2, kP53) DWT2_PV(kSepV, 2, kP53)
                DWT2_MH(kSepH, 0, kU53) DWT2_MV(kSepV, 0, kU53)
                scale(a, e, kZeta53Sq, kZeta53SqInv);
            } else {
                scale(a, e, kZeta53SqInv, kZeta53Sq);
                DWT2_MV(kSepV, 3, -kU53) DWT2_MH(kSepH, 1, -kU53)
                DWT2_PV(kSepV, 1, -kP53) DWT2_PH(kSepH, 0, -kP53)
            }
        } else if constexpr (DIR == kForward) {
            DWT2_PH(kSepH, 3, kAlpha) DWT2_PV(kSepV, 3, kAlpha)
            DWT2_MH(kSepH, 3, kBeta) DWT2_MV(kSepV, 3, kBeta)
            DWT2_PH(kSepH, 2, kGamma) DWT2_PV(kSepV, 2, kGamma)
            DWT2_MH(kSepH, 0, kDelta) DWT2_MV(kSepV, 0, kDelta)
            scale(a, e, kZeta2, kZetaM2);
        } else {
            scale(a, e, kZetaM2, kZeta2);
            DWT2_MV(kSepV, 3, -kDelta) DWT2_MH(kSepH, 3, -kDelta)
            DWT2_PV(kSepV, 3, -kGamma) DWT2_PH(kSepH, 3, -kGamma)
            DWT2_MV(kSepV, 3, -kBeta) DWT2_MH(kSepH, 1, -kBeta)
            DWT2_PV(kSepV, 1, -kAlpha) DWT2_PH(kSepH, 0, -kAlpha)
        }
    } else if constexpr (WAV == kCdf53) {
        if constexpr (DIR == kForward) {
            DWT2_PLUS(kIntFwd, 2, 0.f)
            DWT2_MINUS(kIntFwd, 0, 0.f)
        } else {
            DWT2_MINUS(kIntInv, 1, 0.f)
            DWT2_PLUS(kIntInv, 0, 0.f)
        }
    } else if constexpr (WAV == kCdf53Real) {
        static_assert(DIR != kAdjoint, "the adjoint is implemented for CDF 9/7");
        if constexpr (DIR == kForward) {
            if constexpr (SCH == kSchemeSplit) {
                local_predict(a, e, kP53);
                DWT2_PLUS(kSplit, 2, kP53) local_update(a, e, kU53);
                DWT2_MINUS(kSplit, 0, kU53)
            } else {
                DWT2_PLUS(kFloat, 2, kP53)
                DWT2_MINUS(kFloat, 0, kU53)
            }
            scale(a, e, kZeta53Sq, kZeta53SqInv);
        } else {
            scale(a, e, kZeta53SqInv, kZeta53Sq);
            if constexpr (SCH == kSchemeSplit) {
                DWT2_MINUS(kSplit, 1, -kU53) local_update(a, e, -kU53);
                DWT2_PLUS(kSplit, 0, -kP53) local_predict(a, e, -kP53);
            } else {
                DWT2_MINUS(kFloat, 1, -kU53)
                DWT2_PLUS(kFloat, 0, -kP53)
            }
        }
    } else if constexpr (DIR == kForward) {
        if constexpr (SCH == kSchemeSplit) {
            local_predict(a, e, kAlpha);
            DWT2_PLUS(kSplit, 3, kAlpha) local_update(a, e, kBeta);
            DWT2_MINUS(kSplit, 3, kBeta) local_predict(a, e, kGamma);
            DWT2_PLUS(kSplit, 2, kGamma) local_update(a, e, kDelta);
            DWT2_MINUS(kSplit, 0, kDelta)
        } else {
            DWT2_PLUS(kFloat, 3, kAlpha)
            DWT2_MINUS(kFloat, 3, kBeta)
            DWT2_PLUS(kFloat, 2, kGamma)
            DWT2_MINUS(kFloat, 0, kDelta)
        }
        scale(a, e, kZeta2, kZetaM2);
    } else if constexpr (DIR == kInverse) {
        scale(a, e, kZetaM2, kZeta2);
        if constexpr (SCH == kSchemeSplit) {
            DWT2_MINUS(kSplit, 3, -kDelta) local_update(a, e, -kDelta);
            DWT2_PLUS(kSplit, 3, -kGamma) local_predict(a, e, -kGamma);
            DWT2_MINUS(kSplit, 1, -kBeta) local_update(a, e, -kBeta);
            DWT2_PLUS(kSplit, 0, -kAlpha) local_predict(a, e, -kAlpha);
        } else {
            DWT2_MINUS(kFloat, 3, -kDelta)
            DWT2_PLUS(kFloat, 3, -kGamma)
            DWT2_MINUS(kFloat, 1, -kBeta)
            DWT2_PLUS(kFloat, 0, -kAlpha)
        }
    } else {
        // W^T = T_1^T S_1^T T_2^T S_2^T Z: transposed steps in reverse order;
        // the transpose of an update is predict-shaped and vice versa.
        scale(a, e, kZeta2, kZetaM2);
        DWT2_PLUS(kAdj, 3, kDelta)
        DWT2_MINUS(kAdj, 3, kGamma)
        DWT2_PLUS(kAdj, 2, kBeta)
        DWT2_MINUS(kAdj, 0, kAlpha)
    }
#undef DWT2_PLUS
#undef DWT2_MINUS
#undef DWT2_PH
#undef DWT2_PV
#undef DWT2_MH
#undef DWT2_MV
}

// ---------------------------------------------------------------------------
// global memory access
// ---------------------------------------------------------------------------
// Vector stores of whole output rows are streamed (nontemporal): the
// outputs are not read again by this launch, and the stores of a tile cover
// whole cache lines.  NT = false: an ordinary store, for an LL band that the
// next level of the same transform reads at once.
template <typename T, bool NT = true>
__device__ __forceinline__ void nt_store2(T* p, T a, T b) {
    if constexpr (sizeof(T) == 4) {
        typedef int v2 __attribute__((ext_vector_type(2)));
        v2 q;
        q.x = __builtin_bit_cast(int, a);
        q.y = __builtin_bit_cast(int, b);
        if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v2*>(p));
        else *reinterpret_cast<v2*>(p) = q;
    } else {
        typedef short v2 __attribute__((ext_vector_type(2)));
        v2 q;
        q.x = __builtin_bit_cast(short, a);
        q.y = __builtin_bit_cast(short, b);
        if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v2*>(p));
        else *reinterpret_cast<v2*>(p) = q;
    }
}
template <typename T, bool NT = true>
__device__ __forceinline__ void nt_store4(T* p, T a, T b, T c, T d) {
    if constexpr (sizeof(T) == 4) {
        typedef int v4 __attribute__((ext_vector_type(4)));
        v4 q;
        q.x = __builtin_bit_cast(int, a); q.y = __builtin_bit_cast(int, b);
        q.z = __builtin_bit_cast(int, c); q.w = __builtin_bit_cast(int, d);
        if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v4*>(p));
        else *reinterpret_cast<v4*>(p) = q;
    } else {
        typedef short v4 __attribute__((ext_vector_type(4)));
        v4 q;
        q.x = __builtin_bit_cast(short, a); q.y = __builtin_bit_cast(short, b);
        q.z = __builtin_bit_cast(short, c); q.w = __builtin_bit_cast(short, d);
        if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v4*>(p));
        else *reinterpret_cast<v4*>(p) = q;
    }
}

// Eight 16-bit samples as one 16-byte nontemporal (NT) or ordinary store.
template <typename T, bool NT = true>
__device__ __forceinline__ void nt_store8(T* p, const T (&v)[8]) {
    static_assert(sizeof(T) == 2, "16-bit samples");
    typedef int v4 __attribute__((ext_vector_type(4)));
    v4 q;
    q.x = (int)((unsigned)__builtin_bit_cast(unsigned short, v[0]) | ((unsigned)__builtin_bit_cast(unsigned short, v[1]) << 16));
    q.y = (int)((unsigned)__builtin_bit_cast(unsigned short, v[2]) | ((unsigned)__builtin_bit_cast(unsigned short, v[3]) << 16));
    q.z = (int)((unsigned)__builtin_bit_cast(unsigned short, v[4]) | ((unsigned)__builtin_bit_cast(unsigned short, v[5]) << 16));
    q.w = (int)((unsigned)__builtin_bit_cast(unsigned short, v[6]) | ((unsigned)__builtin_bit_cast(unsigned short, v[7]) << 16));
    if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v4*>(p));
    else *reinterpret_cast<v4*>(p) = q;
}

// One LL sample that a later level of the same persistent launch reads,
// possibly on another XCD: an agent-scope store, which the L2 writes
// through, so the reader sees it after its acquire (an L2 invalidate)
// without the writing tile having to write back its whole L2.
template <typename T>
__device__ __forceinline__ void coherent_store(T* p, typename St<T>::V v) {
    const T t = St<T>::store(v);
    if constexpr (sizeof(T) == 4)
        __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __builtin_bit_cast(uint32_t, t), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_store(reinterpret_cast<uint16_t*>(p), __builtin_bit_cast(uint16_t, t), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

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

template <typename T, bool EDGE, bool NT = true>
__device__ __forceinline__ void store4(T* base, int64_t pitch, int row, int c, int h, int w, bool vec,
                                       typename St<T>::V v0, typename St<T>::V v1,
                                       typename St<T>::V v2, typename St<T>::V v3) {
    if (EDGE && (row >= h || c >= w)) return;
    T* p = base + (int64_t)row * pitch + c;
    if (vec && (!EDGE || c + 3 < w)) {
        nt_store4<T, NT>(p, St<T>::store(v0), St<T>::store(v1), St<T>::store(v2), St<T>::store(v3));
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
        nt_store2(p, St<T>::store(v0), St<T>::store(v1));
    } else {
        p[0] = St<T>::store(v0);
        if (!EDGE || gc + 1 < ncols) p[1] = St<T>::store(v1);
    }
}

// N consecutive samples (blocks gc .. gc+N-1; gc a multiple of N) of one
// subband row with `ncols` columns; outside the row (or !row_ok) read as 0.
template <typename T, bool EDGE, int N>
__device__ __forceinline__ void loadN(const T* rowp, int gc, int ncols, bool row_ok, bool vec,
                                      typename St<T>::V (&v)[N]) {
    using V = typename St<T>::V;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = V(0);
    if (EDGE && (!row_ok || gc < 0 || gc >= ncols)) return;
    const T* p = rowp + gc;
    if (vec && (!EDGE || gc + N - 1 < ncols)) {
        if constexpr (N == 2) {
            const Pack2<T> q = *reinterpret_cast<const Pack2<T>*>(p);
            v[0] = St<T>::load(q.v[0]); v[1] = St<T>::load(q.v[1]);
        } else {
            const Pack4<T> q = *reinterpret_cast<const Pack4<T>*>(p);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = St<T>::load(q.v[i]);
        }
    } else {
        v[0] = St<T>::load(p[0]);
#pragma unroll
        for (int i = 1; i < N; ++i)
            if (!EDGE || gc + i < ncols) v[i] = St<T>::load(p[i]);
    }
}

template <typename T, bool EDGE, int N, bool NT = true>
__device__ __forceinline__ void storeN(T* rowp, int gc, int ncols, bool vec, const typename St<T>::V (&v)[N]) {
    if (EDGE && gc >= ncols) return;
    T* p = rowp + gc;
    if (vec && (!EDGE || gc + N - 1 < ncols)) {
        if constexpr (N == 2) nt_store2<T, NT>(p, St<T>::store(v[0]), St<T>::store(v[1]));
        else nt_store4<T, NT>(p, St<T>::store(v[0]), St<T>::store(v[1]), St<T>::store(v[2]), St<T>::store(v[3]));
    } else {
        p[0] = St<T>::store(v[0]);
#pragma unroll
        for (int i = 1; i < N; ++i)
            if (!EDGE || gc + i < ncols) p[i] = St<T>::store(v[i]);
    }
}

// Semi-vector access for rows that are only 8-byte aligned (even pitches):
// four image samples as two pairs, a subband row segment as pairs when its
// base is even, else sample by sample.  Interior tiles only (no bounds).
template <typename T>
__device__ __forceinline__ void load4_pairs(const T* base, int64_t pitch, int row, int c, typename St<T>::V& v0,
                                            typename St<T>::V& v1, typename St<T>::V& v2,
                                            typename St<T>::V& v3) {
    const T* p = base + (int64_t)row * pitch + c;
    const Pack2<T> q0 = *reinterpret_cast<const Pack2<T>*>(p);
    const Pack2<T> q1 = *reinterpret_cast<const Pack2<T>*>(p + 2);
    v0 = St<T>::load(q0.v[0]); v1 = St<T>::load(q0.v[1]);
    v2 = St<T>::load(q1.v[0]); v3 = St<T>::load(q1.v[1]);
}
template <typename T>
__device__ __forceinline__ void nt_store1(T* p, T a) {
    if constexpr (sizeof(T) == 4) __builtin_nontemporal_store(__builtin_bit_cast(int, a), reinterpret_cast<int*>(p));
    else __builtin_nontemporal_store(__builtin_bit_cast(short, a), reinterpret_cast<short*>(p));
}
template <typename T, int N>
__device__ __forceinline__ void storeN_pairs(T* p, const typename St<T>::V (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; i += 2) nt_store2(p + i, St<T>::store(v[i]), St<T>::store(v[i + 1]));
}

// Load the tile into registers: the core rows of the lane (a) and, in the
// halo lanes, the lane's halo blocks (e).
template <int DIR, typename T, bool EDGE, int BPL, int K>
__device__ __forceinline__ void load_tile(typename St<T>::V (&a)[K][Lay<BPL>::BX], typename St<T>::V (&e)[8],
                                          const LevelParams& P, const Geo& g, const TileGeo<BPL>& tg, int lane) {
    using V = typename St<T>::V;
    const bool vec = EDGE ? P.vec != 0 : true;      // interior tiles run only on aligned images
    const bool halo_lane = lane < 32 && tg.re < K;
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = V(0);
    if constexpr (DIR == kForward) {
        const T* in = static_cast<const T*>(P.in);
        // 16-bit samples, 4 blocks per lane: a lane's 8 samples of an image
        // row are one 16-byte load (rows 16-byte aligned: vec16)
        bool wide = false;
        if constexpr (!EDGE && sizeof(T) == 2 && BPL == 4) {
            wide = P.vec16 != 0;
            if (wide) {
#pragma unroll
                for (int r = 0; r < K; ++r)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const Pack8<T> q = *reinterpret_cast<const Pack8<T>*>(
                            in + (int64_t)(2 * (g.gr0 + r) + h) * P.in_pitch + 2 * g.gcL);
                        // samples 2j, 2j+1 of the row: block j, components 2h, 2h+1
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            a[r][4 * j + 2 * h] = St<T>::load(q.v[2 * j]);
                            a[r][4 * j + 2 * h + 1] = St<T>::load(q.v[2 * j + 1]);
                        }
                    }
            }
        }
        if (!wide) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int row = 2 * (g.gr0 + r);
#pragma unroll
                for (int q = 0; q < BPL / 2; ++q) {
                    const int c = 2 * g.gcL + 4 * q;
                    V* b0 = &a[r][8 * q];
                    load4<T, EDGE>(in, P.in_pitch, row, c, P.h, P.w, vec, b0[0], b0[1], b0[4], b0[5]);
                    load4<T, EDGE>(in, P.in_pitch, row + 1, c, P.h, P.w, vec, b0[2], b0[3], b0[6], b0[7]);
                }
            }
        }
        if (halo_lane) {
            const int row = 2 * tg.gre;
            load4<T, EDGE>(in, P.in_pitch, row, 2 * tg.ge[0], P.h, P.w, vec, e[0], e[1], e[4], e[5]);
            load4<T, EDGE>(in, P.in_pitch, row + 1, 2 * tg.ge[0], P.h, P.w, vec, e[2], e[3], e[6], e[7]);
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
            const T* rows[4] = {ll + gre * P.in_ll_pitch, det + gre * P.in_pitch + g.nEc,
                                det + (g.nEr + gro) * P.in_pitch, det + (g.nEr + gro) * P.in_pitch + g.nEc};
            const int ncols[4] = {g.nEc, g.nOc, g.nEc, g.nOc};
            const bool ok[4] = {rE, rE, rO, rO};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V v[BPL];
                loadN<T, EDGE, BPL>(rows[k], g.gcL, ncols[k], ok[k], vec, v);
#pragma unroll
                for (int b = 0; b < BPL; ++b) a[r][4 * b + k] = v[b];
            }
        }
        if (halo_lane) {
            const int gr = tg.gre;
            const bool rE = gr >= 0 && gr < g.nEr;
            const bool rO = gr >= 0 && gr < g.nOr;
            const int64_t gre = rE ? gr : 0, gro = rO ? gr : 0;
            const T* rows[4] = {ll + gre * P.in_ll_pitch, det + gre * P.in_pitch + g.nEc,
                                det + (g.nEr + gro) * P.in_pitch, det + (g.nEr + gro) * P.in_pitch + g.nEc};
            const int ncols[4] = {g.nEc, g.nOc, g.nEc, g.nOc};
            const bool ok[4] = {rE, rE, rO, rO};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V v[2];
                loadN<T, EDGE, 2>(rows[k], tg.ge[0], ncols[k], ok[k], vec, v);
                e[k] = v[0];
                e[4 + k] = v[1];
            }
        }
    }
}

// Whole-point symmetric extension of a sample index p into [0, n), n >= 2:
// symmetric about both ends, hence periodic with period 2 (n - 1).  |p| is
// folded into one period with a single-precision quotient (the hardware
// reciprocal, within one unit in the last place, a multiply, a conversion)
// and one correction either way: O(1) and a dozen instructions at each
// inlined call site, where an integer modulo is a few dozen and reflecting
// step by step takes about |p| / (n - 1) rounds (the lanes of a tile far
// past a level of a few pixels).  The quotient is off by at most one
// whenever |p| / (2 (n - 1)) < 2^21, which holds for every index a tile
// reaches (at most a tile width past an image of at least 2 pixels).
__device__ __forceinline__ int reflect(int p, int n) {
    if (p >= 0 && p < n) return p;
    const int period = 2 * (n - 1);
    int q = p < 0 ? -p : p;
    q -= (int)((float)q * __builtin_amdgcn_rcpf((float)period)) * period;
    if (q < 0) q += period;
    else if (q >= period) q -= period;
    return q < n ? q : period - q;
}

// Border tiles of the forward and inverse transforms: the tile is loaded
// from the whole-point symmetric extension of the image (forward) or of each
// subband (inverse: the extension that the forward transform of the extended
// image has, i.e. each component sample taken at the reflected pixel
// position), and the fused steps then run without index clamps.  Each step
// keeps the extension symmetric, and every sum a step forms pairs the same
// two values as the clamped step at the same place, so every coefficient
// equals the clamped computation bit for bit.
template <int DIR, typename T, int BPL, int K>
__device__ __forceinline__ void load_tile_mirror(typename St<T>::V (&a)[K][Lay<BPL>::BX], typename St<T>::V (&e)[8],
                                                 const LevelParams& P, const Geo& g, const TileGeo<BPL>& tg,
                                                 int lane) {
    using V = typename St<T>::V;
    const bool vec = P.vec != 0;
    const bool halo_lane = lane < 32 && tg.re < K;
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = V(0);
    if constexpr (DIR == kForward) {
        const T* in = static_cast<const T*>(P.in);
        // component k of block (br, bc) of the extended image
        auto sample = [&](int br, int bc, int k) -> V {
            const int r = reflect(2 * br + (k >> 1), P.h), c = reflect(2 * bc + (k & 1), P.w);
            return St<T>::load(in[(int64_t)r * P.in_pitch + c]);
        };
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int br = g.gr0 + r;
#pragma unroll
            for (int q = 0; q < BPL / 2; ++q) {
                const int c = 2 * g.gcL + 4 * q;          // first pixel column of blocks 2q, 2q+1
                V* b0 = &a[r][8 * q];
                if (vec && c >= 0 && c + 3 < P.w) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int row = reflect(2 * br + h, P.h);
                        load4<T, false>(in, P.in_pitch, row, c, P.h, P.w, true, b0[2 * h], b0[2 * h + 1],
                                        b0[4 + 2 * h], b0[4 + 2 * h + 1]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        b0[k] = sample(br, g.gcL + 2 * q, k);
                        b0[4 + k] = sample(br, g.gcL + 2 * q + 1, k);
                    }
                }
            }
        }
        if (halo_lane) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                e[k] = sample(tg.gre, tg.ge[0], k);
                e[4 + k] = sample(tg.gre, tg.ge[1], k);
            }
        }
    } else {
        const T* ll = static_cast<const T*>(P.in_ll);
        const T* det = static_cast<const T*>(P.in);
        // row base of subband k (0 LL, 1 HL, 2 LH, 3 HH) at component row br
        auto row_of = [&](int k, int br) -> const T* {
            switch (k) {
                case 0: return ll + (int64_t)br * P.in_ll_pitch;
                case 1: return det + (int64_t)br * P.in_pitch + g.nEc;
                case 2: return det + (int64_t)(g.nEr + br) * P.in_pitch;
                default: return det + (int64_t)(g.nEr + br) * P.in_pitch + g.nEc;
            }
        };
        // component k of block (br, bc) of the extended pyramid level
        auto sample = [&](int br, int bc, int k) -> V {
            const int r = (reflect(2 * br + (k >> 1), P.h) - (k >> 1)) >> 1;
            const int c = (reflect(2 * bc + (k & 1), P.w) - (k & 1)) >> 1;
            return St<T>::load(row_of(k, r)[c]);
        };
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int br = g.gr0 + r;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ncols = (k & 1) ? g.nOc : g.nEc;
                if (vec && g.gcL >= 0 && g.gcL + BPL - 1 < ncols) {
                    const int rr = (reflect(2 * br + (k >> 1), P.h) - (k >> 1)) >> 1;
                    V v[BPL];
                    loadN<T, false, BPL>(row_of(k, rr), g.gcL, ncols, true, true, v);
#pragma unroll
                    for (int b = 0; b < BPL; ++b) a[r][4 * b + k] = v[b];
                } else {
#pragma unroll
                    for (int b = 0; b < BPL; ++b) a[r][4 * b + k] = sample(br, g.gcL + b, k);
                }
            }
        }
        if (halo_lane) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                e[k] = sample(tg.gre, tg.ge[0], k);
                e[4 + k] = sample(tg.gre, tg.ge[1], k);
            }
        }
    }
}

// Store the core of the tile: the core blocks of every lane, halo rows
// dropped.  Forward, interior tiles of 4-byte samples: one subband after the
// other (the rows of LL, then HL, LH, HH), which suits the memory system
// slightly better than interleaving the four quadrants row by row.
template <int DIR, typename T, bool EDGE, int NW, int BPL, int K, bool LLC = false, bool LLX = false>
__device__ __forceinline__ void store_tile(typename St<T>::V (&a)[K][Lay<BPL>::BX], const LevelParams& P,
                                           const Geo& g, int wv) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    const bool vec = EDGE ? P.vec != 0 : true;      // interior tiles run only on aligned images
    if constexpr (DIR == kForward) {
        T* ll = static_cast<T*>(P.out_ll);
        T* det = static_cast<T*>(P.out);
        constexpr bool kBySubband = !EDGE && sizeof(T) == 4;
#pragma unroll
        for (int k0 = 0; k0 < (kBySubband ? 4 : 1); ++k0)
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int tr = wv * K + r;        // row within the tile
                if (tr < kHalo || tr >= kHalo + kCoreBY) continue;
                const int gr = g.gr0 + r;
                if (EDGE && gr >= g.nEr) continue;
#pragma unroll
                for (int k = (kBySubband ? k0 : 0); k < (kBySubband ? k0 + 1 : 4); ++k) {
                    if (EDGE && k >= 2 && gr >= g.nOr) continue;
                    V v[BPL];
#pragma unroll
                    for (int b = 0; b < BPL; ++b) v[b] = a[r][4 * b + k];
                    T* row = k == 0 ? ll + (int64_t)gr * P.out_ll_pitch
                           : k == 1 ? det + (int64_t)gr * P.out_pitch + g.nEc
                           : k == 2 ? det + (int64_t)(g.nEr + gr) * P.out_pitch
                                    : det + (int64_t)(g.nEr + gr) * P.out_pitch + g.nEc;
                    if (LLX && k == 0) {
#pragma unroll
                        for (int b = 0; b < BPL; ++b)
                            if (!EDGE || g.gcL + b < g.nEc) coherent_store<T>(row + g.gcL + b, v[b]);
                    } else if (LLC && k == 0) {
                        storeN<T, EDGE, BPL, false>(row, g.gcL, g.nEc, vec, v);
                    } else {
                        storeN<T, EDGE, BPL>(row, g.gcL, (k & 1) ? g.nOc : g.nEc, vec, v);
                    }
                }
            }
    } else {
        T* img = static_cast<T*>(P.out);
        bool wide = false;
        if constexpr (!EDGE && sizeof(T) == 2 && BPL == 4) wide = P.vec16 != 0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int tr = wv * K + r;
            if (tr < kHalo || tr >= kHalo + kCoreBY) continue;
            const int gr = g.gr0 + r;
            if (EDGE && gr >= g.nEr) continue;
            if constexpr (!EDGE && sizeof(T) == 2 && BPL == 4) {
                if (wide) {
                    // 16-bit samples, 4 blocks per lane: one 16-byte store per image row
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        T o[8];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            o[2 * j] = St<T>::store(a[r][4 * j + 2 * h]);
                            o[2 * j + 1] = St<T>::store(a[r][4 * j + 2 * h + 1]);
                        }
                        nt_store8<T, !LLC>(img + (int64_t)(2 * gr + h) * P.out_pitch + 2 * g.gcL, o);
                    }
                    continue;
                }
            }
#pragma unroll
            for (int q = 0; q < BPL / 2; ++q) {
                const int c = 2 * g.gcL + 4 * q;
                const V* b0 = &a[r][8 * q];
                store4<T, EDGE, !LLC>(img, P.out_pitch, 2 * gr, c, P.h, P.w, vec, b0[0], b0[1], b0[4], b0[5]);
                store4<T, EDGE, !LLC>(img, P.out_pitch, 2 * gr + 1, c, P.h, P.w, vec, b0[2], b0[3], b0[6], b0[7]);
            }
        }
    }
}

// A subband row segment whose first sample sits at an odd element offset
// (HL, HH rows when the low-pass width is odd): the pairs start one sample
// later, each lane pairing its last sample with the next lane's first (DPP);
// lane 0 stores the tile's first sample alone, lane 63 its last.
template <typename T, int N>
__device__ __forceinline__ void storeN_shifted(T* p, const typename St<T>::V (&v)[N], int lane) {
    using V = typename St<T>::V;
    const V next = from_right(v[0]);
#pragma unroll
    for (int i = 1; i + 1 < N; i += 2) nt_store2(p + i, St<T>::store(v[i]), St<T>::store(v[i + 1]));
    if (lane < kLanes - 1) nt_store2(p + N - 1, St<T>::store(v[N - 1]), St<T>::store(next));
    else nt_store1(p + N - 1, St<T>::store(v[N - 1]));
    if (lane == 0) nt_store1(p, St<T>::store(v[0]));
}

// The load counterpart of storeN_shifted: a subband row segment whose first
// sample sits at an odd element offset is read as pairs starting one sample
// later; each lane's first sample is the previous lane's last pair's second
// (DPP), lane 0 reads its first sample alone.  The last lane's last pair
// reaches one sample into the next tile (inside the image for interior
// tiles).
template <typename T, int N>
__device__ __forceinline__ void loadN_shifted(const T* p, typename St<T>::V (&v)[N], int lane) {
    using V = typename St<T>::V;
    V last;
#pragma unroll
    for (int i = 1; i < N; i += 2) {
        const Pack2<T> q = *reinterpret_cast<const Pack2<T>*>(p + i);
        v[i] = St<T>::load(q.v[0]);
        if (i + 1 < N) v[i + 1] = St<T>::load(q.v[1]);
        else last = St<T>::load(q.v[1]);
    }
    const V first = from_left(last);
    if (lane == 0) v[0] = St<T>::load(p[0]);
    else v[0] = first;
}
template <typename T, int N>
__device__ __forceinline__ void loadN_pairs(const T* p, typename St<T>::V (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; i += 2) {
        const Pack2<T> q = *reinterpret_cast<const Pack2<T>*>(p + i);
        v[i] = St<T>::load(q.v[0]);
        v[i + 1] = St<T>::load(q.v[1]);
    }
}

// Interior tile of an image whose rows are only 8-byte aligned (vec8): the
// accesses of load_tile / store_tile as sample pairs; HL, HH rows starting at
// an odd offset (odd low-pass width) as shifted pairs.
template <int DIR, typename T, int BPL, int K>
__device__ __forceinline__ void load_tile_semi(typename St<T>::V (&a)[K][Lay<BPL>::BX], typename St<T>::V (&e)[8],
                                               const LevelParams& P, const Geo& g, const TileGeo<BPL>& tg,
                                               int lane) {
    using V = typename St<T>::V;
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = V(0);
    const bool halo_lane = lane < 32 && tg.re < K;
    if constexpr (DIR == kForward) {
        const T* in = static_cast<const T*>(P.in);
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int row = 2 * (g.gr0 + r);
#pragma unroll
            for (int q = 0; q < BPL / 2; ++q) {
                const int c = 2 * g.gcL + 4 * q;
                V* b0 = &a[r][8 * q];
                load4_pairs<T>(in, P.in_pitch, row, c, b0[0], b0[1], b0[4], b0[5]);
                load4_pairs<T>(in, P.in_pitch, row + 1, c, b0[2], b0[3], b0[6], b0[7]);
            }
        }
        if (halo_lane) {
            const int row = 2 * tg.gre;
            load4_pairs<T>(in, P.in_pitch, row, 2 * tg.ge[0], e[0], e[1], e[4], e[5]);
            load4_pairs<T>(in, P.in_pitch, row + 1, 2 * tg.ge[0], e[2], e[3], e[6], e[7]);
        }
    } else {
        const T* ll = static_cast<const T*>(P.in_ll);
        const T* det = static_cast<const T*>(P.in);
        const bool hi_pairs = (g.nEc & 1) == 0;   // HL, HH rows start at column nEc
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int64_t gr = g.gr0 + r;
            const T* rows[4] = {ll + gr * P.in_ll_pitch, det + gr * P.in_pitch + g.nEc,
                                det + (g.nEr + gr) * P.in_pitch, det + (g.nEr + gr) * P.in_pitch + g.nEc};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V v[BPL];
                if ((k & 1) && !hi_pairs) loadN_shifted<T, BPL>(rows[k] + g.gcL, v, lane);
                else loadN_pairs<T, BPL>(rows[k] + g.gcL, v);
#pragma unroll
                for (int b = 0; b < BPL; ++b) a[r][4 * b + k] = v[b];
            }
        }
        if (halo_lane) {
            const int64_t gr = tg.gre;
            const T* rows[4] = {ll + gr * P.in_ll_pitch, det + gr * P.in_pitch + g.nEc,
                                det + (g.nEr + gr) * P.in_pitch, det + (g.nEr + gr) * P.in_pitch + g.nEc};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T* p = rows[k] + tg.ge[0];
                e[k] = St<T>::load(p[0]);
                e[4 + k] = St<T>::load(p[1]);
            }
        }
    }
}

template <int DIR, typename T, int NW, int BPL, int K, bool LLX = false>
__device__ __forceinline__ void store_tile_semi(typename St<T>::V (&a)[K][Lay<BPL>::BX], const LevelParams& P,
                                                const Geo& g, int wv, int lane) {
    using V = typename St<T>::V;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    if constexpr (DIR == kForward) {
        T* ll = static_cast<T*>(P.out_ll);
        T* det = static_cast<T*>(P.out);
        const bool hi_pairs = (g.nEc & 1) == 0;   // HL, HH rows start at column nEc
        constexpr bool kBySubband = sizeof(T) == 4;
#pragma unroll
        for (int k0 = 0; k0 < (kBySubband ? 4 : 1); ++k0)
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const int tr = wv * K + r;
                if (tr < kHalo || tr >= kHalo + kCoreBY) continue;
                const int gr = g.gr0 + r;
#pragma unroll
                for (int k = (kBySubband ? k0 : 0); k < (kBySubband ? k0 + 1 : 4); ++k) {
                    V v[BPL];
#pragma unroll
                    for (int b = 0; b < BPL; ++b) v[b] = a[r][4 * b + k];
                    T* row = k == 0 ? ll + (int64_t)gr * P.out_ll_pitch
                           : k == 1 ? det + (int64_t)gr * P.out_pitch + g.nEc
                           : k == 2 ? det + (int64_t)(g.nEr + gr) * P.out_pitch
                                    : det + (int64_t)(g.nEr + gr) * P.out_pitch + g.nEc;
                    if (LLX && k == 0) {
#pragma unroll
                        for (int b = 0; b < BPL; ++b) coherent_store<T>(row + g.gcL + b, v[b]);
                    } else if ((k & 1) && !hi_pairs) {
                        storeN_shifted<T, BPL>(row + g.gcL, v, lane);
                    } else {
                        storeN_pairs<T, BPL>(row + g.gcL, v);
                    }
                }
            }
    } else {
        T* img = static_cast<T*>(P.out);
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int tr = wv * K + r;
            if (tr < kHalo || tr >= kHalo + kCoreBY) continue;
            const int64_t gr = g.gr0 + r;
#pragma unroll
            for (int q = 0; q < BPL / 2; ++q) {
                const int c = 2 * g.gcL + 4 * q;
                const V* b0 = &a[r][8 * q];
                T* p0 = img + (2 * gr) * P.out_pitch + c;
                T* p1 = p0 + P.out_pitch;
                nt_store2(p0, St<T>::store(b0[0]), St<T>::store(b0[1]));
                nt_store2(p0 + 2, St<T>::store(b0[4]), St<T>::store(b0[5]));
                nt_store2(p1, St<T>::store(b0[2]), St<T>::store(b0[3]));
                nt_store2(p1 + 2, St<T>::store(b0[6]), St<T>::store(b0[7]));
            }
        }
    }
}

// One tile (tx, ty) of one level: load, the fused steps, store.  The LDS
// belongs to the calling work-group.
// SEMI: interior tiles of images with 8-byte aligned rows (vec8) take the
// semi-vector path instead of the border path.
template <int DIR, int WAV, typename T, int SCH, int NW, int K, int BPL, bool SEMI = false, bool LLC = false,
          bool LLX = false>
__device__ __forceinline__ void tile_body(const LevelParams& P, int tx, int ty,
                                          TileLds<typename St<T>::V, NW, BPL, K>& lds, int lane, int wv) {
    using V = typename St<T>::V;
    using L = Lay<BPL>;
    constexpr int kCoreBY = NW * K - 2 * kHalo;
    Geo g;
    g.nEr = (P.h + 1) >> 1; g.nOr = P.h >> 1;
    g.nEc = (P.w + 1) >> 1; g.nOc = P.w >> 1;
    const int cb0 = tx * L::CORE_BX, rb0 = ty * kCoreBY;
    g.gcL = cb0 + BPL * lane;
    g.gr0 = rb0 - kHalo + wv * K;
    TileGeo<BPL> tg;
#pragma unroll
    for (int b = 0; b < BPL; ++b) tg.gc[b] = g.gcL + b;
    tg.re = lane & 15;
    tg.gre = g.gr0 + tg.re;
    tg.ge[0] = (lane & 16) ? cb0 + L::CORE_BX : cb0 - kHalo;
    tg.ge[1] = tg.ge[0] + 1;
    // Interior tile: every loaded block has all four components, no
    // neighbour index of the core's dependency cone needs clamping, and (the
    // image's rows being aligned) every access is a full vector (SEMI: a
    // pair of samples).
    const bool inside = rb0 - kHalo >= 0 && cb0 - kHalo >= 0 &&
                        rb0 + kCoreBY + kHalo <= g.nOr && cb0 + L::CORE_BX + kHalo <= g.nOc;
    const bool interior = (SEMI ? P.vec8 != 0 : P.vec != 0) && inside;
    V a[K][L::BX];
    V e[8];
    if (interior) {
        if constexpr (SEMI) {
            load_tile_semi<DIR, T, BPL>(a, e, P, g, tg, lane);
            run<DIR, WAV, false, SCH, NW, BPL>(a, e, lds, lane, wv, g, tg);
            store_tile_semi<DIR, T, NW, BPL, K, LLX>(a, P, g, wv, lane);
        } else {
            load_tile<DIR, T, false, BPL>(a, e, P, g, tg, lane);
            run<DIR, WAV, false, SCH, NW, BPL>(a, e, lds, lane, wv, g, tg);
            store_tile<DIR, T, false, NW, BPL, K, LLC, LLX>(a, P, g, wv);
        }
    } else if constexpr (DIR != kAdjoint) {
        // border tile: symmetric extension at load time, unclamped steps
        // (the split applies to interior tiles only)
        load_tile_mirror<DIR, T, BPL>(a, e, P, g, tg, lane);
        run<DIR, WAV, false, SCH == kSchemeSplit ? kSchemeFused : SCH, NW, BPL>(a, e, lds, lane, wv, g, tg);
        store_tile<DIR, T, true, NW, BPL, K, false, LLX>(a, P, g, wv);
    } else {
        // the adjoint's border weights are not a symmetric extension
        load_tile<DIR, T, true, BPL>(a, e, P, g, tg, lane);
        run<DIR, WAV, true, kSchemeFused, NW, BPL>(a, e, lds, lane, wv, g, tg);
        store_tile<DIR, T, true, NW, BPL>(a, P, g, wv);
    }
}

// The level parameters of plane `pl` of a plane batch (buffers offset by
// the plane strides).
// Selects, not branches: a buffer the direction does not use stays null.
// Pointer arithmetic (not integer casts) keeps the buffers in the global
// address space for the compiler, so accesses stay global_load /
// global_store rather than flat ones.
template <typename T, typename P_>
__device__ __forceinline__ P_* plane_ptr(P_* p, int pl, int64_t stride) {
    return p ? static_cast<P_*>(static_cast<T*>(const_cast<void*>(static_cast<const void*>(p))) +
                                (int64_t)pl * stride)
             : p;
}
template <typename T>
__device__ __forceinline__ LevelParams plane_params(const LevelParams& P, int pl) {
    LevelParams Q = P;
    Q.in = plane_ptr<T>(P.in, pl, P.in_ps);
    Q.in_ll = plane_ptr<T>(P.in_ll, pl, P.in_ll_ps);
    Q.out = plane_ptr<T>(P.out, pl, P.out_ps);
    Q.out_ll = plane_ptr<T>(P.out_ll, pl, P.out_ll_ps);
    return Q;
}

// Every field of the level parameters is taken into SGPRs here, before the
// first branch and before any value derived from them: the scalar loads of
// the kernel arguments then go out together and cost one memory round trip
// per wave, where loads issued at each field's first use (after the tile
// index arithmetic, inside the plane-offset code) cost three or four.
__device__ __forceinline__ void fetch_params(const LevelParams& P) {
    asm volatile("" ::"s"(P.in), "s"(P.in_pitch), "s"(P.in_ll), "s"(P.in_ll_pitch), "s"(P.out), "s"(P.out_pitch),
                 "s"(P.out_ll), "s"(P.out_ll_pitch), "s"(P.h), "s"(P.w), "s"(P.tiles_x), "s"(P.tiles_y), "s"(P.vec),
                 "s"(P.in_ps), "s"(P.in_ll_ps), "s"(P.out_ps), "s"(P.out_ll_ps), "s"(P.planes), "s"(P.vec8),
                 "s"(P.vec16));
}

template <int DIR, int WAV, typename T, int SCH, int NW, int K, int BPL, bool SEMI, bool LLC = false>
__global__ void __launch_bounds__(NW * kLanes) level_kernel(LevelParams P) {
    using V = typename St<T>::V;
    __shared__ TileLds<V, NW, BPL, K> lds;
    const int lane = threadIdx.x & (kLanes - 1);
    // the wave index is uniform: keep it (and every row address) in SGPRs
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    fetch_params(P);
    // Work-groups are dealt round-robin over the 8 XCDs.  XCD x takes chunks
    // x, x + 8, x + 16, ... of kRemapRows whole tile rows: horizontal halo
    // re-reads stay in that XCD's L2 (and vertical ones within a chunk),
    // while the 8 XCDs work on adjacent chunks, so the image is swept by
    // one narrow window (8 chunks tall) rather than 8 distant ones.
    // The tiles of a plane batch form one list, plane after plane, dealt
    // the same way: small planes do not each round up to 8 chunks.
    const int nt = P.tiles_x * P.tiles_y;
    const int chunk = kRemapRows * P.tiles_x;
    const int j = (int)(blockIdx.x >> 3);
    const int g = ((j / chunk) * 8 + (int)(blockIdx.x & 7)) * chunk + j % chunk;
    if (g >= nt * P.planes) return;               // uniform over the work-group
    const int pl = g / nt;
    const int t = g - pl * nt;
    const int ty = t / P.tiles_x;
    const int tx = t - ty * P.tiles_x;
    tile_body<DIR, WAV, T, SCH, NW, K, BPL, SEMI, LLC>(plane_params<T>(P, pl), tx, ty, lds, lane, wv);
}

// ===========================================================================
// Streaming kernel: one wave64 marches down a column strip of the image.
//
// The strip is 128 blocks wide (2 per lane, a 2-block halo on each side, as
// in the tile kernel); the wave walks a segment of block rows top to bottom.
// Each iteration brings one new block row into a small register window and
// advances every fused step by one row: a predict-shaped step on row r needs
// row r+1 at the previous stage, so it runs one row behind that stage; an
// update-shaped step on row r needs row r-1, which is already done, so it
// runs in the same row as the previous stage.  For CDF 9/7 forward the steps
// T, S, T, S run on rows i-1, i-1, i-2, i-2 when row i arrives; the row
// leaving the window is final and stored.  The value an update-shaped step
// reads from the row above must be taken before that row was itself updated:
// it is saved just before the update.  Horizontal neighbours come from the
// adjacent lane (DPP); there is no LDS and no barrier, and loads run a few
// rows ahead of the computation.  A segment re-reads only the 2 block rows
// above and below it.
// ===========================================================================
struct StepSpec {
    bool plus;    // predict-shaped (reads the row below) or update-shaped
    int kind;     // Kind of the fused step
    float c;      // its coefficient
    int after;    // split: constant part applied to the same row right after
                  // (0 none, 1 predict-local, 2 update-local)
    float ca;     // coefficient of that constant part
};

template <int DIR, int WAV, bool SPLIT> struct Prog;

template <bool SPLIT> struct Prog<kForward, kCdf97, SPLIT> {
    static constexpr int N = 4;
    static constexpr StepSpec kSteps[N] = {
        {true, SPLIT ? kSplit : kFloat, kAlpha, SPLIT ? 2 : 0, kBeta},
        {false, SPLIT ? kSplit : kFloat, kBeta, SPLIT ? 1 : 0, kGamma},
        {true, SPLIT ? kSplit : kFloat, kGamma, SPLIT ? 2 : 0, kDelta},
        {false, SPLIT ? kSplit : kFloat, kDelta, 0, 0.f}};
    static constexpr int kPreLocal = SPLIT ? 1 : 0;     // constant part of the first predict
    static constexpr float kPreLocalC = kAlpha;
    static constexpr bool kPreScale = false;
    static constexpr float kPre0 = 1.f, kPre3 = 1.f;
    static constexpr bool kPostScale = true;
    static constexpr float kPost0 = kZeta2, kPost3 = kZetaM2;
};
template <bool SPLIT> struct Prog<kInverse, kCdf97, SPLIT> {
    static constexpr int N = 4;
    static constexpr StepSpec kSteps[N] = {
        {false, SPLIT ? kSplit : kFloat, -kDelta, SPLIT ? 2 : 0, -kDelta},
        {true, SPLIT ? kSplit : kFloat, -kGamma, SPLIT ? 1 : 0, -kGamma},
        {false, SPLIT ? kSplit : kFloat, -kBeta, SPLIT ? 2 : 0, -kBeta},
        {true, SPLIT ? kSplit : kFloat, -kAlpha, SPLIT ? 1 : 0, -kAlpha}};
    static constexpr int kPreLocal = 0;
    static constexpr float kPreLocalC = 0.f;
    static constexpr bool kPreScale = true;
    static constexpr float kPre0 = kZetaM2, kPre3 = kZeta2;
    static constexpr bool kPostScale = false;
    static constexpr float kPost0 = 1.f, kPost3 = 1.f;
};
template <bool SPLIT> struct Prog<kAdjoint, kCdf97, SPLIT> {
    static constexpr int N = 4;
    static constexpr StepSpec kSteps[N] = {
        {true, kAdj, kDelta, 0, 0.f}, {false, kAdj, kGamma, 0, 0.f},
        {true, kAdj, kBeta, 0, 0.f}, {false, kAdj, kAlpha, 0, 0.f}};
    static constexpr int kPreLocal = 0;
    static constexpr float kPreLocalC = 0.f;
    static constexpr bool kPreScale = true;
    static constexpr float kPre0 = kZeta2, kPre3 = kZetaM2;
    static constexpr bool kPostScale = false;
    static constexpr float kPost0 = 1.f, kPost3 = 1.f;
};
template <bool SPLIT> struct Prog<kForward, kCdf53Real, SPLIT> {
    static constexpr int N = 2;
    static constexpr StepSpec kSteps[N] = {
        {true, SPLIT ? kSplit : kFloat, kP53, SPLIT ? 2 : 0, kU53},
        {false, SPLIT ? kSplit : kFloat, kU53, 0, 0.f}};
    static constexpr int kPreLocal = SPLIT ? 1 : 0;
    static constexpr float kPreLocalC = kP53;
    static constexpr bool kPreScale = false;
    static constexpr float kPre0 = 1.f, kPre3 = 1.f;
    static constexpr bool kPostScale = true;
    static constexpr float kPost0 = kZeta53Sq, kPost3 = kZeta53SqInv;
};
template <bool SPLIT> struct Prog<kInverse, kCdf53Real, SPLIT> {
    static constexpr int N = 2;
    static constexpr StepSpec kSteps[N] = {
        {false, SPLIT ? kSplit : kFloat, -kU53, SPLIT ? 2 : 0, -kU53},
        {true, SPLIT ? kSplit : kFloat, -kP53, SPLIT ? 1 : 0, -kP53}};
    static constexpr int kPreLocal = 0;
    static constexpr float kPreLocalC = 0.f;
    static constexpr bool kPreScale = true;
    static constexpr float kPre0 = kZeta53SqInv, kPre3 = kZeta53Sq;
    static constexpr bool kPostScale = false;
    static constexpr float kPost0 = 1.f, kPost3 = 1.f;
};
template <bool SPLIT> struct Prog<kForward, kCdf53, SPLIT> {
    static constexpr int N = 2;
    static constexpr StepSpec kSteps[N] = {{true, kIntFwd, 0.f, 0, 0.f}, {false, kIntFwd, 0.f, 0, 0.f}};
    static constexpr int kPreLocal = 0;
    static constexpr float kPreLocalC = 0.f;
    static constexpr bool kPreScale = false;
    static constexpr float kPre0 = 1.f, kPre3 = 1.f;
    static constexpr bool kPostScale = false;
    static constexpr float kPost0 = 1.f, kPost3 = 1.f;
};
template <bool SPLIT> struct Prog<kInverse, kCdf53, SPLIT> {
    static constexpr int N = 2;
    static constexpr StepSpec kSteps[N] = {{false, kIntInv, 0.f, 0, 0.f}, {true, kIntInv, 0.f, 0, 0.f}};
    static constexpr int kPreLocal = 0;
    static constexpr float kPreLocalC = 0.f;
    static constexpr bool kPreScale = false;
    static constexpr float kPre0 = 1.f, kPre3 = 1.f;
    static constexpr bool kPostScale = false;
    static constexpr float kPost0 = 1.f, kPost3 = 1.f;
};

// Rows behind the newest row at which step k runs.
template <class PR>
constexpr int step_lag(int k) {
    int lag = 0;
    for (int j = 0; j <= k; ++j) lag += PR::kSteps[j].plus ? 1 : 0;
    return lag;
}
template <class PR>
constexpr int max_lag() { return step_lag<PR>(PR::N - 1); }

// Predict-shaped step on one row (cur) reading the row below (dn).
template <int KIND, bool EX, bool EY, typename V>
__device__ __forceinline__ void plus_row(V (&cur)[8], const V (&dn)[8], int gcL, int gr, const Geo& g, float c) {
    const V rrow = from_right(cur[0]);
    const V rR2 = from_right(cur[2]);
    const V dRR = from_right(dn[0]);
    plus_block<KIND, EX, EY>(cur[0], cur[1], cur[2], cur[3], cur[4], cur[6], dn[0], dn[1], dn[4], gcL, gr, g, c);
    plus_block<KIND, EX, EY>(cur[4], cur[5], cur[6], cur[7], rrow, rR2, dn[4], dn[5], dRR, gcL + 1, gr, g, c);
}

// Update-shaped step on one row reading x2 and x3 of the row above (up2, up3:
// L then R), both taken just before that row's own update: later steps of
// the pipeline (the constant predict part of the split) may change them.
template <int KIND, bool EX, bool EY, typename V>
__device__ __forceinline__ void minus_row(V (&cur)[8], const V (&up)[4], int gcL, int gr,
                                          const Geo& g, float c) {
    const V lL1 = from_left(cur[5]);
    const V lL3 = from_left(cur[7]);
    const V uLL3 = from_left(up[3]);
    minus_block<KIND, EX, EY>(cur[4], cur[5], cur[6], cur[7], cur[1], cur[3], up[1], up[3], up[2],
                              gcL + 1, gr, g, c);
    minus_block<KIND, EX, EY>(cur[0], cur[1], cur[2], cur[3], lL1, lL3, up[0], up[2], uLL3, gcL, gr, g, c);
}

template <typename V>
__device__ __forceinline__ void local_row(V (&r)[8], int what, float c) {
#pragma unroll
    for (int b = 0; b < 8; b += 4) {
        if (what == 1) {
            r[b + 1] = fmaf(c, r[b + 0], r[b + 1]);
            r[b + 3] = fmaf(c, r[b + 2], r[b + 3]);
            r[b + 2] = fmaf(c, r[b + 0], r[b + 2]);
            r[b + 3] = fmaf(c, r[b + 1], r[b + 3]);
        } else if (what == 2) {
            r[b + 0] = fmaf(c, r[b + 1], r[b + 0]);
            r[b + 2] = fmaf(c, r[b + 3], r[b + 2]);
            r[b + 0] = fmaf(c, r[b + 2], r[b + 0]);
            r[b + 1] = fmaf(c, r[b + 3], r[b + 1]);
        }
    }
}

// All steps of one iteration (newest row i), step k onward.
template <class PR, int k, bool EX, bool EY, typename V, int NWIN>
__device__ __forceinline__ void steps_from(V (&win)[NWIN][8], V (&sv)[PR::N][4], int i, int gcL, const Geo& g) {
    if constexpr (k < PR::N) {
        constexpr StepSpec st = PR::kSteps[k];
        constexpr int lag = step_lag<PR>(k);
        const int gr = i - lag;
        if constexpr (st.plus) {
            plus_row<st.kind, EX, EY>(win[lag], win[lag - 1], gcL, gr, g, st.c);
        } else {
            // x2, x3 of this row before its update, for the next row's update
            const V s0 = win[lag][2], s1 = win[lag][6], s2 = win[lag][3], s3 = win[lag][7];
            minus_row<st.kind, EX, EY>(win[lag], sv[k], gcL, gr, g, st.c);
            sv[k][0] = s0;
            sv[k][1] = s1;
            sv[k][2] = s2;
            sv[k][3] = s3;
        }
        if constexpr (st.after != 0) local_row(win[lag], st.after, st.ca);
        steps_from<PR, k + 1, EX, EY>(win, sv, i, gcL, g);
    }
}

// Raw block row `row` of the input into r (zeros outside the image).
template <int DIR, typename T>
__device__ __forceinline__ void stream_load(typename St<T>::V (&r)[8], const LevelParams& P, const Geo& g, int row) {
    using V = typename St<T>::V;
    const bool vec = P.vec != 0;
    if constexpr (DIR == kForward) {
        const T* in = static_cast<const T*>(P.in);
        load4<T, true>(in, P.in_pitch, 2 * row, 2 * g.gcL, P.h, P.w, vec, r[0], r[1], r[4], r[5]);
        load4<T, true>(in, P.in_pitch, 2 * row + 1, 2 * g.gcL, P.h, P.w, vec, r[2], r[3], r[6], r[7]);
    } else {
        const T* ll = static_cast<const T*>(P.in_ll);
        const T* det = static_cast<const T*>(P.in);
        const bool rE = row >= 0 && row < g.nEr;
        const bool rO = row >= 0 && row < g.nOr;
        const int64_t gre = rE ? row : 0, gro = rO ? row : 0;
        load2<T, true>(ll + gre * P.in_ll_pitch, g.gcL, g.nEc, rE, vec, r[0], r[4]);
        load2<T, true>(det + gre * P.in_pitch + g.nEc, g.gcL, g.nOc, rE, vec, r[1], r[5]);
        load2<T, true>(det + (g.nEr + gro) * P.in_pitch, g.gcL, g.nEc, rO, vec, r[2], r[6]);
        load2<T, true>(det + (g.nEr + gro) * P.in_pitch + g.nEc, g.gcL, g.nOc, rO, vec, r[3], r[7]);
        (void)sizeof(V);
    }
}

// Final block row gr to the output (core lanes only).
template <int DIR, typename T, class PR>
__device__ __forceinline__ void stream_store(const typename St<T>::V (&r)[8], const LevelParams& P, const Geo& g,
                                             int gr) {
    const bool vec = P.vec != 0;
    if constexpr (DIR == kForward) {
        T* ll = static_cast<T*>(P.out_ll);
        T* det = static_cast<T*>(P.out);
        using V = typename St<T>::V;
        V l0 = r[0], l1 = r[4], h0 = r[3], h1 = r[7];
        if constexpr (PR::kPostScale) {
            l0 *= PR::kPost0; l1 *= PR::kPost0;
            h0 *= PR::kPost3; h1 *= PR::kPost3;
        }
        store2<T, true>(ll + (int64_t)gr * P.out_ll_pitch, g.gcL, g.nEc, vec, l0, l1);
        store2<T, true>(det + (int64_t)gr * P.out_pitch + g.nEc, g.gcL, g.nOc, vec, r[1], r[5]);
        if (gr < g.nOr) {
            store2<T, true>(det + (int64_t)(g.nEr + gr) * P.out_pitch, g.gcL, g.nEc, vec, r[2], r[6]);
            store2<T, true>(det + (int64_t)(g.nEr + gr) * P.out_pitch + g.nEc, g.gcL, g.nOc, vec, h0, h1);
        }
    } else {
        T* img = static_cast<T*>(P.out);
        const int c = 2 * g.gcL;
        store4<T, true>(img, P.out_pitch, 2 * gr, c, P.h, P.w, vec, r[0], r[1], r[4], r[5]);
        store4<T, true>(img, P.out_pitch, 2 * gr + 1, c, P.h, P.w, vec, r[2], r[3], r[6], r[7]);
    }
}

template <int DIR, int WAV, typename T, bool SPLIT, bool EX, int PF>
__device__ __forceinline__ void stream_segment(const LevelParams& P, const Geo& g, int lane, int s0, int s1) {
    using V = typename St<T>::V;
    using PR = Prog<DIR, WAV, SPLIT>;
    constexpr int LAGMAX = max_lag<PR>();
    constexpr int NWIN = LAGMAX + 1;
    const bool core_lane = lane >= kHalo / 2 && lane < kLanes - kHalo / 2;
    const int i0 = s0 - kHalo;
    const int i1 = s1 + LAGMAX;                   // one past the last iteration
    V win[NWIN][8];
    V sv[PR::N][4];
    V ring[PF][8];
#pragma unroll
    for (int j = 0; j < NWIN; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) win[j][q] = V(0);
#pragma unroll
    for (int j = 0; j < PR::N; ++j) sv[j][0] = sv[j][1] = sv[j][2] = sv[j][3] = V(0);
#pragma unroll
    for (int u = 0; u < PF; ++u) stream_load<DIR, T>(ring[u], P, g, i0 + u < i1 ? i0 + u : -1);

    for (int base = i0; base < i1; base += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = base + u;
            if (i < i1) {
#pragma unroll
                for (int j = NWIN - 1; j > 0; --j)
#pragma unroll
                    for (int q = 0; q < 8; ++q) win[j][q] = win[j - 1][q];
#pragma unroll
                for (int q = 0; q < 8; ++q) win[0][q] = ring[u][q];
                stream_load<DIR, T>(ring[u], P, g, i + PF < i1 ? i + PF : -1);
                if constexpr (PR::kPreScale) {
                    win[0][0] *= PR::kPre0; win[0][4] *= PR::kPre0;
                    win[0][3] *= PR::kPre3; win[0][7] *= PR::kPre3;
                }
                if constexpr (PR::kPreLocal != 0) local_row(win[0], PR::kPreLocal, PR::kPreLocalC);
                // rows whose neighbour indices need clamping: the first and the last rows of the image
                const bool ey = i < 3 || i >= g.nOr - 1;
                if (ey) steps_from<PR, 0, EX, true>(win, sv, i, g.gcL, g);
                else steps_from<PR, 0, EX, false>(win, sv, i, g.gcL, g);
                const int gr = i - LAGMAX;
                if (core_lane && gr >= s0 && gr < s1) stream_store<DIR, T, PR>(win[LAGMAX], P, g, gr);
            }
        }
    }
}

template <int DIR, int WAV, typename T, bool SPLIT, int W, int PF>
__global__ void __launch_bounds__(W * kLanes) stream_kernel(LevelParams P0) {
    const LevelParams P = plane_params<T>(P0, (int)blockIdx.y);
    const int lane = threadIdx.x & (kLanes - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    // consecutive work-groups of one XCD take vertically adjacent segments,
    // so the rows a segment re-reads from its neighbours are in that XCD's L2
    const int nt = P.tiles_x * P.tiles_y;
    const int per = (nt + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (t >= nt) return;
    const int gx = t / P.tiles_y;
    const int gy = t - gx * P.tiles_y;
    Geo g;
    g.nEr = (P.h + 1) >> 1; g.nOr = P.h >> 1;
    g.nEc = (P.w + 1) >> 1; g.nOc = P.w >> 1;
    const int nsx = (g.nEc + kStreamCoreBX - 1) / kStreamCoreBX;
    const int sx = gx * W + wv;
    if (sx >= nsx) return;                        // waves are independent: no barrier follows
    const int cb0 = sx * kStreamCoreBX;
    g.gcL = cb0 - kHalo + 2 * lane;
    g.gr0 = 0;
    const int s0 = gy * P.seg_rows;
    const int s1 = min(s0 + P.seg_rows, g.nEr);
    const bool ix = cb0 - kHalo >= 0 && cb0 + kStreamCoreBX + kHalo <= g.nOc;
    const bool iy = s0 - kHalo >= 0 && s1 + kHalo <= g.nOr;
    if (ix) {
        if (SPLIT && iy) stream_segment<DIR, WAV, T, SPLIT, false, PF>(P, g, lane, s0, s1);
        else stream_segment<DIR, WAV, T, false, false, PF>(P, g, lane, s0, s1);
    } else {
        stream_segment<DIR, WAV, T, false, true, PF>(P, g, lane, s0, s1);
    }
}


}  // namespace kern
}  // namespace dwt2
