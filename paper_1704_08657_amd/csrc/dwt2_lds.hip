// LDS-plane tile kernel: any step program over the four polyphase planes of
// a tile held in LDS.  Used for the schemes and wavelets the register tile
// kernel does not cover -- the non-separable polyconvolution N_{P,U}
// (Section "Proposed Schemes"), the DD 13/7 wavelet with its four-tap steps
// (Section "Evaluation") -- and, on the same footing, the fused and separable
// lifting schemes, so that the schemes can be compared in one kernel design.
//
// This is the on-chip-memory design the paper's OpenCL kernels follow: a
// work-group loads its tile plus a halo into on-chip memory as the quadruple
// of polyphase components, then runs one calculation step after the other,
// each a 2-D stencil over the planes followed by one barrier, and writes the
// tile's core.  Here:
//   * the planes live in LDS twice (source and destination of a step), so a
//     step reads only values of the previous step and needs one barrier;
//   * a step computes every block of its output region, which shrinks by the
//     step's reach from one step to the next, so the tile's halo is the sum
//     of the reaches (two blocks per side for CDF 9/7, three for DD 13/7);
//   * tiles touching the image border load the whole-point symmetric
//     extension (forward: the reflected pixel; inverse: each subband sample
//     at its reflected pixel position) and then run the same steps, as the
//     register tile kernel does;
//   * the CDF steps of the fused and separable schemes evaluate each block
//     with the register tile kernel's block formulas, so their results are
//     bit-identical to that kernel's.
// Work-groups are dealt over the 8 XCDs in chunks of whole tile rows, as in
// the register tile kernel.
#include "dwt2_kernels.inl"

namespace dwt2 {
namespace kern {
namespace lds {

constexpr int kThreads = 256;

// A 1-D lifting filter: taps c[0 .. n-1] at offsets lo .. lo + n - 1 (offset
// k reads sample m + k).
struct Filt {
    int lo, n;
    float c[4];
};
constexpr Filt neg(Filt f) {
    Filt g = f;
    for (int i = 0; i < 4; ++i) g.c[i] = -f.c[i];
    return g;
}
constexpr int hi(Filt f) { return f.lo + f.n - 1; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int imax(int a, int b) { return a > b ? a : b; }

// CDF filters in the library's convention: P(z) = p (1 + z), U(z) = u (1 + z^-1).
constexpr Filt cdfP(float p) { return Filt{0, 2, {p, p, 0.f, 0.f}}; }
constexpr Filt cdfU(float u) { return Filt{-1, 2, {u, u, 0.f, 0.f}}; }
// Deslauriers-Dubuc 13/7: the 4-point interpolating predict and its update.
constexpr Filt kDdP{-1, 4, {1.f / 16, -9.f / 16, -9.f / 16, 1.f / 16}};
constexpr Filt kDdU{-2, 4, {-1.f / 32, 9.f / 32, 9.f / 32, -1.f / 32}};
// DD 13/7 scaling: the predict removes constants, so the low-pass DC gain
// after lifting is 1 and zeta = sqrt(2): LL * 2, HH * 1/2.
constexpr float kZetaDdSq = 2.0f, kZetaDdSqInv = 0.5f;

// Step kinds: fused predict T_P / update S_U, the polyconvolution N_{P,U}
// and its inverse, and the four separable 1-D steps.
enum StepKind : int { kT, kS, kN, kNinv, kTH, kTV, kSH, kSV };
struct Step {
    int kind;
    Filt P, U;     // kT, kTH, kTV: P; kS, kSH, kSV: U; kN, kNinv: both
    bool cdf;      // two-tap CDF filters: evaluated with the register kernel's block formulas
};

// Reach of a step: the offsets it reads along each axis.
struct Reach { int xlo, xhi, ylo, yhi; };
constexpr Reach reach_of(Step s) {
    const Filt P = s.P, U = s.U;
    // V = P U + 1 reads offsets P.lo + U.lo .. hi(P) + hi(U) and 0
    const int vlo = imin(0, P.lo + U.lo), vhi = imax(0, hi(P) + hi(U));
    switch (s.kind) {
        case kT: return {P.lo, hi(P), P.lo, hi(P)};
        case kS: return {U.lo, hi(U), U.lo, hi(U)};
        case kN:
        case kNinv: {
            const int lo = imin(vlo, imin(P.lo, U.lo)), h = imax(vhi, imax(hi(P), hi(U)));
            return {lo, h, lo, h};
        }
        case kTH: return {P.lo, hi(P), 0, 0};
        case kTV: return {0, 0, P.lo, hi(P)};
        case kSH: return {U.lo, hi(U), 0, 0};
        default: return {0, 0, U.lo, hi(U)};
    }
}

// The step programs.  Forward: the steps, then LL * s0 and HH * s3 at the
// store; inverse: LL * s0 and HH * s3 at the load, then the steps.
template <int DIR, int WAV, int SCH> struct Prog;

template <int WAV> struct Pairs;
template <> struct Pairs<kCdf97> {
    static constexpr int K = 2;
    static constexpr Filt P[2] = {cdfP(kAlpha), cdfP(kGamma)};
    static constexpr Filt U[2] = {cdfU(kBeta), cdfU(kDelta)};
    static constexpr bool cdf = true;
    static constexpr float z2 = kZeta2, z2inv = kZetaM2;
};
template <> struct Pairs<kCdf53Real> {
    static constexpr int K = 1;
    static constexpr Filt P[1] = {cdfP(kP53)};
    static constexpr Filt U[1] = {cdfU(kU53)};
    static constexpr bool cdf = true;
    static constexpr float z2 = kZeta53Sq, z2inv = kZeta53SqInv;
};
template <> struct Pairs<kDd137> {
    static constexpr int K = 1;
    static constexpr Filt P[1] = {kDdP};
    static constexpr Filt U[1] = {kDdU};
    static constexpr bool cdf = false;
    static constexpr float z2 = kZetaDdSq, z2inv = kZetaDdSqInv;
};


template <int WAV, int SCH> struct Prog<kForward, WAV, SCH> {
    using W = Pairs<WAV>;
    static constexpr int N = SCH == kSchemePolyconv ? W::K : SCH == kSchemeSeparable ? 4 * W::K : 2 * W::K;
    static constexpr Step step(int i) {
        if (SCH == kSchemePolyconv) return Step{kN, W::P[i], W::U[i], W::cdf};
        if (SCH == kSchemeSeparable) {
            const int k = i / 4, j = i % 4;
            const int kinds[4] = {kTH, kTV, kSH, kSV};
            return Step{kinds[j], W::P[k], W::U[k], W::cdf};
        }
        return Step{(i & 1) ? kS : kT, W::P[i / 2], W::U[i / 2], W::cdf};
    }
    static constexpr float s0 = W::z2, s3 = W::z2inv;
};
template <int WAV, int SCH> struct Prog<kInverse, WAV, SCH> {
    using W = Pairs<WAV>;
    static constexpr int N = Prog<kForward, WAV, SCH>::N;
    // the forward steps in reverse order, each undone: the fused and
    // separable steps with negated filters (their horizontal and vertical
    // factors commute), N_{P,U} by its inverse
    static constexpr Step step(int i) {
        const Step f = Prog<kForward, WAV, SCH>::step(N - 1 - i);
        if (f.kind == kN) return Step{kNinv, f.P, f.U, f.cdf};
        return Step{f.kind, neg(f.P), neg(f.U), f.cdf};
    }
    static constexpr float s0 = W::z2inv, s3 = W::z2;
};

// Output region of step i in tile coordinates (the loaded region is
// [0, RH) x [0, RW)): each step drops the blocks whose operands fall outside
// the previous step's region.
struct Region { int x0, x1, y0, y1; };
template <class PR>
constexpr Region region_after(int i, int RW, int RH) {
    Region r{0, RW, 0, RH};
    for (int k = 0; k <= i; ++k) {
        const Reach a = reach_of(PR::step(k));
        r.x0 -= a.xlo; r.x1 -= a.xhi; r.y0 -= a.ylo; r.y1 -= a.yhi;
    }
    return r;
}
// Halo (blocks per side) the program needs: the largest shrink over the
// four sides.
template <class PR>
constexpr int halo_of() {
    int l = 0, r = 0, t = 0, b = 0;
    for (int k = 0; k < PR::N; ++k) {
        const Reach a = reach_of(PR::step(k));
        l -= a.xlo; r += a.xhi; t -= a.ylo; b += a.yhi;
    }
    return imax(imax(l, r), imax(t, b));
}

template <int RH, int RW> struct Planes {
    float p[2][4][RH][RW];
};

// ---------------------------------------------------------------------------
// one block of one step: read the source planes around (n, m), return the
// four outputs
// ---------------------------------------------------------------------------
template <int RH, int RW> struct At {
    const float (&q)[4][RH][RW];
    int n, m;
    __device__ float operator()(int c, int dn, int dm) const { return q[c][n + dn][m + dm]; }
};

// sum_j f.c[j] x(dn, f.lo + j) along m / along n
template <class X>
__device__ __forceinline__ float hf(const X& x, int c, int dn, Filt f) {
    float s = f.c[0] * x(c, dn, f.lo);
#pragma unroll
    for (int j = 1; j < f.n; ++j) s = fmaf(f.c[j], x(c, dn, f.lo + j), s);
    return s;
}
template <class X>
__device__ __forceinline__ float vf(const X& x, int c, int dm, Filt f) {
    float s = f.c[0] * x(c, f.lo, dm);
#pragma unroll
    for (int i = 1; i < f.n; ++i) s = fmaf(f.c[i], x(c, f.lo + i, dm), s);
    return s;
}

template <int KIND, class X>
__device__ __forceinline__ void step_block(const X& x, const Step st, float (&o)[4]) {
    const Filt P = st.P, U = st.U;
    float x0 = x(0, 0, 0), x1 = x(1, 0, 0), x2 = x(2, 0, 0), x3 = x(3, 0, 0);
    if constexpr (KIND == kT || KIND == kTH || KIND == kTV) {
        if (st.cdf) {
            // the register tile kernel's block formula (bit-identical
            // results); a 1-D step reads only the operands of its own axis,
            // within the step's reach
            const Geo g{};
            const float x0R = KIND != kTV ? x(0, 0, 1) : 0.f, x2R = KIND != kTV ? x(2, 0, 1) : 0.f;
            const float x0D = KIND != kTH ? x(0, 1, 0) : 0.f, x1D = KIND != kTH ? x(1, 1, 0) : 0.f;
            const float x0DR = KIND == kT ? x(0, 1, 1) : 0.f;
            plus_block<KIND == kT ? kFloat : KIND == kTH ? kSepH : kSepV, false, false>(
                x0, x1, x2, x3, x0R, x2R, x0D, x1D, x0DR, 0, 0, g, P.c[0]);
        } else if constexpr (KIND == kT) {
            // x1 += P x0, x2 += P* x0, x3 += P P* x0 + P* x1 + P x2
            float pp = 0.f;
#pragma unroll
            for (int i = 0; i < P.n; ++i) pp = fmaf(P.c[i], hf(x, 0, P.lo + i, P), pp);
            x3 = x3 + pp + vf(x, 1, 0, P) + hf(x, 2, 0, P);
            x1 = x1 + hf(x, 0, 0, P);
            x2 = x2 + vf(x, 0, 0, P);
        } else if constexpr (KIND == kTH) {
            x1 = x1 + hf(x, 0, 0, P);
            x3 = x3 + hf(x, 2, 0, P);
        } else {
            x2 = x2 + vf(x, 0, 0, P);
            x3 = x3 + vf(x, 1, 0, P);
        }
    } else if constexpr (KIND == kS || KIND == kSH || KIND == kSV) {
        if (st.cdf) {
            const Geo g{};
            const float x1l = KIND != kSV ? x(1, 0, -1) : 0.f, x3l = KIND != kSV ? x(3, 0, -1) : 0.f;
            const float x2u = KIND != kSH ? x(2, -1, 0) : 0.f, x3u = KIND != kSH ? x(3, -1, 0) : 0.f;
            const float x3ul = KIND == kS ? x(3, -1, -1) : 0.f;
            minus_block<KIND == kS ? kFloat : KIND == kSH ? kSepH : kSepV, false, false>(
                x0, x1, x2, x3, x1l, x3l, x2u, x3u, x3ul, 0, 0, g, U.c[0]);
        } else if constexpr (KIND == kS) {
            // x0 += U x1 + U* x2 + U U* x3, x1 += U* x3, x2 += U x3
            float uu = 0.f;
#pragma unroll
            for (int i = 0; i < U.n; ++i) uu = fmaf(U.c[i], hf(x, 3, U.lo + i, U), uu);
            x0 = x0 + hf(x, 1, 0, U) + vf(x, 2, 0, U) + uu;
            x1 = x1 + vf(x, 3, 0, U);
            x2 = x2 + hf(x, 3, 0, U);
        } else if constexpr (KIND == kSH) {
            x0 = x0 + hf(x, 1, 0, U);
            x2 = x2 + hf(x, 3, 0, U);
        } else {
            x0 = x0 + vf(x, 2, 0, U);
            x1 = x1 + vf(x, 3, 0, U);
        }
    } else {
        // N_{P,U} = N^V N^H with the pair matrix [[V, U], [P, 1]] per axis,
        // V = P U + 1 (Section "Proposed Schemes"); its inverse with
        // [[1, -U], [-P, V]].  The horizontal factor of row dn is applied to
        // the pairs (x0, x1) and (x2, x3), the vertical factor to its results:
        // every output is computed from this step's inputs only.
        // V a at (dn, 0) along m: a + sum_j U_j sum_k P_k a(j + k)
        auto Vh = [&](int c, int dn) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < U.n; ++j) s = fmaf(U.c[j], hf(x, c, dn, Filt{P.lo + U.lo + j, P.n, {P.c[0], P.c[1], P.c[2], P.c[3]}}), s);
            return x(c, dn, 0) + s;
        };
        if constexpr (KIND == kN) {
            // horizontal results of row dn: e = V a + U b, o = P a + b
            auto E = [&](int a, int dn) { return Vh(a, dn) + hf(x, a + 1, dn, U); };
            auto O = [&](int a, int dn) { return hf(x, a, dn, P) + x(a + 1, dn, 0); };
            // vertical: x0' = V* E0 + U* E2, x1' = V* O0 + U* O2,
            //           x2' = P* E0 + E2,    x3' = P* O0 + O2
            float vE = 0.f, vO = 0.f, uE = 0.f, uO = 0.f, pE = 0.f, pO = 0.f;
#pragma unroll
            for (int j = 0; j < U.n; ++j) {
                float sE = 0.f, sO = 0.f;
#pragma unroll
                for (int k = 0; k < P.n; ++k) {
                    sE = fmaf(P.c[k], E(0, U.lo + j + P.lo + k), sE);
                    sO = fmaf(P.c[k], O(0, U.lo + j + P.lo + k), sO);
                }
                vE = fmaf(U.c[j], sE, vE);
                vO = fmaf(U.c[j], sO, vO);
                uE = fmaf(U.c[j], E(2, U.lo + j), uE);
                uO = fmaf(U.c[j], O(2, U.lo + j), uO);
            }
#pragma unroll
            for (int k = 0; k < P.n; ++k) {
                pE = fmaf(P.c[k], E(0, P.lo + k), pE);
                pO = fmaf(P.c[k], O(0, P.lo + k), pO);
            }
            x0 = E(0, 0) + vE + uE;
            x1 = O(0, 0) + vO + uO;
            x2 = pE + E(2, 0);
            x3 = pO + O(2, 0);
        } else {
            // horizontal results of row dn: e = a - U b, o = -P a + V b
            auto E = [&](int a, int dn) { return x(a, dn, 0) - hf(x, a + 1, dn, U); };
            auto O = [&](int a, int dn) { return Vh(a + 1, dn) - hf(x, a, dn, P); };
            // vertical: x0' = E0 - U* E2, x1' = O0 - U* O2,
            //           x2' = -P* E0 + V* E2, x3' = -P* O0 + V* O2
            float vE = 0.f, vO = 0.f, uE = 0.f, uO = 0.f, pE = 0.f, pO = 0.f;
#pragma unroll
            for (int j = 0; j < U.n; ++j) {
                float sE = 0.f, sO = 0.f;
#pragma unroll
                for (int k = 0; k < P.n; ++k) {
                    sE = fmaf(P.c[k], E(2, U.lo + j + P.lo + k), sE);
                    sO = fmaf(P.c[k], O(2, U.lo + j + P.lo + k), sO);
                }
                vE = fmaf(U.c[j], sE, vE);
                vO = fmaf(U.c[j], sO, vO);
                uE = fmaf(U.c[j], E(2, U.lo + j), uE);
                uO = fmaf(U.c[j], O(2, U.lo + j), uO);
            }
#pragma unroll
            for (int k = 0; k < P.n; ++k) {
                pE = fmaf(P.c[k], E(0, P.lo + k), pE);
                pO = fmaf(P.c[k], O(0, P.lo + k), pO);
            }
            x0 = E(0, 0) - uE;
            x1 = O(0, 0) - uO;
            x2 = E(2, 0) + vE - pE;
            x3 = O(2, 0) + vO - pO;
        }
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// Step i of the program over its output region, source buffer i & 1,
// destination buffer (i + 1) & 1, then the step's barrier.
template <class PR, int I, int RH, int RW>
__device__ __forceinline__ void run_steps(Planes<RH, RW>& L, int tid) {
    if constexpr (I < PR::N) {
        constexpr Step st = PR::step(I);
        constexpr Region r = region_after<PR>(I, RW, RH);
        constexpr int w = r.x1 - r.x0, h = r.y1 - r.y0;
        static_assert(w > 0 && h > 0, "tile too small for the program's reach");
        const float (&src)[4][RH][RW] = L.p[I & 1];
        float (&dst)[4][RH][RW] = L.p[(I + 1) & 1];
        for (int idx = tid; idx < w * h; idx += kThreads) {
            const int n = r.y0 + idx / w, m = r.x0 + idx % w;
            float o[4];
            step_block<st.kind>(At<RH, RW>{src, n, m}, st, o);
#pragma unroll
            for (int c = 0; c < 4; ++c) dst[c][n][m] = o[c];
        }
        __syncthreads();
        run_steps<PR, I + 1, RH, RW>(L, tid);
    }
}

// ---------------------------------------------------------------------------
// global memory
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void load_pair(const T* p, bool pair, float& a, float& b) {
    if (pair) {
        const Pack2<T> q = *reinterpret_cast<const Pack2<T>*>(p);
        a = St<T>::load(q.v[0]);
        b = St<T>::load(q.v[1]);
    } else {
        a = St<T>::load(p[0]);
        b = St<T>::load(p[1]);
    }
}

// Forward load: pixel rows 2 (rb0 - H) ... of the image into the planes of
// buffer 0 (block (n, m) of the tile = image block (rb0 - H + n, cb0 - H + m));
// outside the image the whole-point symmetric extension.
template <typename T, int H, int RH, int RW>
__device__ __forceinline__ void load_fwd(Planes<RH, RW>& L, const LevelParams& P, int rb0, int cb0, bool inside,
                                         int tid) {
    const T* in = static_cast<const T*>(P.in);
    const int r0 = 2 * (rb0 - H), c0 = 2 * (cb0 - H);
    const bool pair = P.vec8 != 0;
    for (int idx = tid; idx < 2 * RH * RW; idx += kThreads) {
        const int pr = idx / RW, bc = idx - pr * RW;
        const int R = r0 + pr, C = c0 + 2 * bc;
        float a, b;
        if (inside) {
            load_pair<T>(in + (int64_t)R * P.in_pitch + C, pair, a, b);
        } else {
            const T* row = in + (int64_t)reflect(R, P.h) * P.in_pitch;
            a = St<T>::load(row[reflect(C, P.w)]);
            b = St<T>::load(row[reflect(C + 1, P.w)]);
        }
        const int q = (pr & 1) * 2;
        L.p[0][q][pr >> 1][bc] = a;
        L.p[0][q + 1][pr >> 1][bc] = b;
    }
}

// Inverse load: the four subbands of the pyramid level into buffer 0, each
// sample outside its subband taken at its reflected pixel position; LL and
// HH scaled.
template <typename T, int H, int RH, int RW>
__device__ __forceinline__ void load_inv(Planes<RH, RW>& L, const LevelParams& P, int rb0, int cb0, bool inside,
                                         float s0, float s3, int tid) {
    const T* ll = static_cast<const T*>(P.in_ll);
    const T* det = static_cast<const T*>(P.in);
    const int nEr = (P.h + 1) >> 1, nEc = (P.w + 1) >> 1;
    for (int idx = tid; idx < 4 * RH * RW; idx += kThreads) {
        const int k = idx / (RH * RW);
        const int rem = idx - k * (RH * RW);
        const int n = rem / RW, m = rem - n * RW;
        const int pr = k >> 1, pc = k & 1;
        int gr = rb0 - H + n, gc = cb0 - H + m;
        if (!inside) {
            gr = (reflect(2 * gr + pr, P.h) - pr) >> 1;
            gc = (reflect(2 * gc + pc, P.w) - pc) >> 1;
        }
        const T* src = k == 0 ? ll + (int64_t)gr * P.in_ll_pitch
                     : k == 1 ? det + (int64_t)gr * P.in_pitch + nEc
                     : k == 2 ? det + (int64_t)(nEr + gr) * P.in_pitch
                              : det + (int64_t)(nEr + gr) * P.in_pitch + nEc;
        float v = St<T>::load(src[gc]);
        if (k == 0) v *= s0;
        if (k == 3) v *= s3;
        L.p[0][k][n][m] = v;
    }
}

// Forward store: the core of buffer B (tile blocks [H, H + CY) x [H, H + CX))
// into the four subbands, LL and HH scaled; blocks past a subband's extent
// are dropped.
template <typename T, int H, int CX, int CY, int RH, int RW>
__device__ __forceinline__ void store_fwd(const float (&q)[4][RH][RW], const LevelParams& P, int rb0, int cb0,
                                          float s0, float s3, int tid) {
    T* ll = static_cast<T*>(P.out_ll);
    T* det = static_cast<T*>(P.out);
    const int nEr = (P.h + 1) >> 1, nOr = P.h >> 1, nEc = (P.w + 1) >> 1, nOc = P.w >> 1;
    for (int idx = tid; idx < 4 * CY * CX; idx += kThreads) {
        const int k = idx / (CY * CX);
        const int rem = idx - k * (CY * CX);
        const int n = rem / CX, m = rem - n * CX;
        const int gr = rb0 + n, gc = cb0 + m;
        if (gr >= ((k & 2) ? nOr : nEr) || gc >= ((k & 1) ? nOc : nEc)) continue;
        float v = q[k][H + n][H + m];
        if (k == 0) v *= s0;
        if (k == 3) v *= s3;
        T* dst = k == 0 ? ll + (int64_t)gr * P.out_ll_pitch
               : k == 1 ? det + (int64_t)gr * P.out_pitch + nEc
               : k == 2 ? det + (int64_t)(nEr + gr) * P.out_pitch
                        : det + (int64_t)(nEr + gr) * P.out_pitch + nEc;
        nt_store1(dst + gc, St<T>::store(v));
    }
}

// Inverse store: the core of buffer B as image pixels (pairs along a row).
template <typename T, int H, int CX, int CY, int RH, int RW>
__device__ __forceinline__ void store_inv(const float (&q)[4][RH][RW], const LevelParams& P, int rb0, int cb0,
                                          int tid) {
    T* img = static_cast<T*>(P.out);
    const bool pair = P.vec8 != 0;
    for (int idx = tid; idx < 2 * CY * CX; idx += kThreads) {
        const int pr = idx / CX, m = idx - pr * CX;
        const int R = 2 * rb0 + pr, C = 2 * (cb0 + m);
        if (R >= P.h || C >= P.w) continue;
        const int k = (pr & 1) * 2;
        const float a = q[k][H + (pr >> 1)][H + m], b = q[k + 1][H + (pr >> 1)][H + m];
        T* p = img + (int64_t)R * P.out_pitch + C;
        if (C + 1 < P.w) {
            if (pair) nt_store2(p, St<T>::store(a), St<T>::store(b));
            else { nt_store1(p, St<T>::store(a)); nt_store1(p + 1, St<T>::store(b)); }
        } else {
            nt_store1(p, St<T>::store(a));
        }
    }
}

template <int DIR, int WAV, int SCH, typename T, int CX, int CY>
__global__ void __launch_bounds__(kThreads) lds_kernel(LevelParams P0) {
    using PR = Prog<DIR, WAV, SCH>;
    constexpr int H = halo_of<PR>();
    constexpr int RH = CY + 2 * H, RW = CX + 2 * H;
    static_assert(sizeof(Planes<RH, RW>) <= 64 * 1024, "LDS of one work-group");
    __shared__ Planes<RH, RW> L;
    const int tid = threadIdx.x;
    // XCD remap of the tile list (all planes), as in the register tile kernel
    const int nt = P0.tiles_x * P0.tiles_y;
    const int chunk = kRemapRows * P0.tiles_x;
    const int j = (int)(blockIdx.x >> 3);
    const int g = ((j / chunk) * 8 + (int)(blockIdx.x & 7)) * chunk + j % chunk;
    if (g >= nt * P0.planes) return;              // uniform over the work-group
    const int pl = g / nt;
    const int t = g - pl * nt;
    const int ty = t / P0.tiles_x;
    const int tx = t - ty * P0.tiles_x;
    const LevelParams P = plane_params<T>(P0, pl);
    const int rb0 = ty * CY, cb0 = tx * CX;
    // every loaded pixel (forward) or subband sample (inverse) inside the image
    const int nOr = P.h >> 1, nOc = P.w >> 1;
    const bool inside = rb0 - H >= 0 && cb0 - H >= 0 && rb0 + CY + H <= nOr && cb0 + CX + H <= nOc;
    if constexpr (DIR == kForward) load_fwd<T, H>(L, P, rb0, cb0, inside, tid);
    else load_inv<T, H>(L, P, rb0, cb0, inside, PR::s0, PR::s3, tid);
    __syncthreads();
    run_steps<PR, 0>(L, tid);
    if constexpr (DIR == kForward) store_fwd<T, H, CX, CY>(L.p[PR::N & 1], P, rb0, cb0, PR::s0, PR::s3, tid);
    else store_inv<T, H, CX, CY>(L.p[PR::N & 1], P, rb0, cb0, tid);
}

template <int DIR, int WAV, int SCH, typename T, int CX, int CY>
hipError_t launch_t(const LevelParams& p, int planes, hipStream_t s) {
    const int64_t nt = (int64_t)p.tiles_x * p.tiles_y;
    const int64_t chunk = (int64_t)kRemapRows * p.tiles_x;
    const int64_t limit = 0x7fffffff - 8 * chunk;
    if (nt < 1 || nt > limit) return hipErrorInvalidConfiguration;
    const int64_t per = limit / nt;
    for (int64_t p0 = 0; p0 < planes; p0 += per) {
        LevelParams q = p;
        q.planes = (int32_t)(planes - p0 < per ? planes - p0 : per);
        if (p0 > 0) {
            if (q.in) q.in = static_cast<const T*>(q.in) + p0 * q.in_ps;
            if (q.in_ll) q.in_ll = static_cast<const T*>(q.in_ll) + p0 * q.in_ll_ps;
            if (q.out) q.out = static_cast<T*>(q.out) + p0 * q.out_ps;
            if (q.out_ll) q.out_ll = static_cast<T*>(q.out_ll) + p0 * q.out_ll_ps;
        }
        const int64_t grid = (nt * q.planes + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
        hipLaunchKernelGGL((lds_kernel<DIR, WAV, SCH, T, CX, CY>), dim3((unsigned)grid), dim3(kThreads), 0, s, q);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int DIR, int WAV, int SCH, typename T>
hipError_t launch_cfg(int cfg, const LevelParams& p, int planes, hipStream_t s) {
    static_assert(kNumConfigs == 10 && kConfigs[8].algo == kAlgoLds && kConfigs[9].algo == kAlgoLds,
                  "LDS-plane configurations 8 and 9");
    switch (cfg) {
        case 8: return launch_t<DIR, WAV, SCH, T, kConfigs[8].cx, kConfigs[8].cy>(p, planes, s);
        case 9: return launch_t<DIR, WAV, SCH, T, kConfigs[9].cx, kConfigs[9].cy>(p, planes, s);
    }
    return hipErrorInvalidValue;
}

template <int DIR, int WAV, typename T>
hipError_t launch_sch(Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    switch (sch) {
        case kSchemeFused: return launch_cfg<DIR, WAV, kSchemeFused, T>(cfg, p, planes, s);
        case kSchemeSeparable: return launch_cfg<DIR, WAV, kSchemeSeparable, T>(cfg, p, planes, s);
        case kSchemePolyconv:
            // one step per lifting pair: a scheme for wavelets of several pairs
            if constexpr (Pairs<WAV>::K > 1) return launch_cfg<DIR, WAV, kSchemePolyconv, T>(cfg, p, planes, s);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int DIR, int WAV>
hipError_t launch_dt(Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    switch (dt) {
        case kF32: return launch_sch<DIR, WAV, float>(sch, cfg, p, planes, s);
        case kBF16: return launch_sch<DIR, WAV, __hip_bfloat16>(sch, cfg, p, planes, s);
        case kF16: return launch_sch<DIR, WAV, __half>(sch, cfg, p, planes, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DIR>
hipError_t launch_wav(Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes, hipStream_t s) {
    switch (wav) {
        case kCdf97: return launch_dt<DIR, kCdf97>(dt, sch, cfg, p, planes, s);
        case kCdf53Real: return launch_dt<DIR, kCdf53Real>(dt, sch, cfg, p, planes, s);
        case kDd137: return launch_dt<DIR, kDd137>(dt, sch, cfg, p, planes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lds
}  // namespace kern

hipError_t launch_lds(Direction dir, Wavelet wav, Dtype dt, Scheme sch, int cfg, const LevelParams& p, int planes,
                      hipStream_t s) {
    if (p.tiles_x <= 0 || p.tiles_y <= 0 || planes <= 0) return hipSuccess;
    switch (dir) {
        case kForward: return kern::lds::launch_wav<kForward>(wav, dt, sch, cfg, p, planes, s);
        case kInverse: return kern::lds::launch_wav<kInverse>(wav, dt, sch, cfg, p, planes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dwt2
