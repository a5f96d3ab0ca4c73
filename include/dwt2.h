/*
 * dwt2.h -- C ABI of a 2-D discrete wavelet transform for AMD Instinct MI355X
 * (gfx950), computed with the non-separable lifting scheme of Barina, Kula,
 * Matysek and Zemcik, "Accelerating Discrete Wavelet Transforms on Parallel
 * Architectures" (WSCG 2017).
 *
 * What is computed (Section "Background"): one scale splits an image into the
 * quadruple of polyphase components x0 = X[2n][2m], x1 = X[2n][2m+1],
 * x2 = X[2n+1][2m], x3 = X[2n+1][2m+1] and maps them by K pairs of lifting
 * steps, eq. (2).  The kernels apply each pair as the two fused spatial steps
 * of Section "Proposed Schemes",
 *     T_P : x1 += P x0, x2 += P* x0, x3 += P P* x0 + P* x1 + P x2
 *     S_U : x0 += U x1 + U* x2 + U U* x3, x1 += U* x3, x2 += U x3
 * with one work-group barrier per step.  With DWT2_FLAG_SPLIT the constant
 * parts P0, U0 run as barrier-free separable lifting and only P1, U1 stay in
 * the fused step (Section "Optimization Approach").  DWT2_FLAG_SEPARABLE runs
 * the separable lifting scheme the paper compares with (one barrier per 1-D
 * step), DWT2_FLAG_FACTORED the fused steps evaluated as their 1-D factors.
 * Wavelets: CDF 9/7 and the real-valued CDF 5/3 (float storage), and the
 * reversible integer CDF 5/3.
 *
 * Conventions (the paper leaves them open; the library fixes them):
 *   - Output layout: Mallat pyramid in an H x W array.  Level l transforms the
 *     LL of level l-1 (ceil halving).  For a level of size h x w with
 *     he = ceil(h/2), we = ceil(w/2): LL = [0,he) x [0,we), HL (x1, high
 *     horizontally) = [0,he) x [we,w), LH (x2) = [he,h) x [0,we),
 *     HH (x3) = [he,h) x [we,w).
 *   - Borders: whole-point symmetric extension (X[-k] = X[k],
 *     X[N-1+k] = X[N-1-k]) per axis, the only boundary supported.
 *   - CDF 9/7: Daubechies-Sweldens lifting constants, then LL * zeta^2,
 *     HH * zeta^-2 (HL, LH unscaled), zeta = 1.1496043988602418, so that a
 *     constant image c gives LL = 2c per level.  Arithmetic is FP32 for every
 *     storage type; BF16/FP16 values are rounded to nearest-even on every
 *     store (intermediate LL levels included).
 *   - Reversible CDF 5/3 (int32 only): odd -= floor((e[m] + e[m+1]) / 2),
 *     even += floor((o[m-1] + o[m] + 2) / 4), in the order T^H, T^V, S^H, S^V
 *     of the separable scheme; exact integer arithmetic.  Pixels must satisfy
 *     |x| < 2^28 (not checked on the device).
 *
 * Memory and streams: every pointer is a device pointer owned by the caller.
 * The library never allocates, frees or synchronises on these calls; all work
 * is enqueued on `stream` (a hipStream_t; NULL is the default stream) and the
 * call returns once it is enqueued.  src and dst must not overlap; the
 * workspace must not overlap either.  Pitches are in elements.
 *
 * Errors: every argument check runs on the host before any HIP call; on an
 * error the call returns a negative dwt2_status, enqueues nothing and leaves
 * dst untouched.  DWT2_E_HIP reports a HIP runtime error at launch; its text
 * is returned by dwt2_last_hip_error() (thread-local).
 */
#ifndef DWT2_H
#define DWT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DWT2_OK = 0,
    DWT2_E_NULL = -1,       /* a required pointer is NULL                       */
    DWT2_E_SHAPE = -2,      /* height or width < 2 (or > 2^30)                  */
    DWT2_E_LEVELS = -3,     /* levels < 1 or > dwt2_max_levels(height, width)   */
    DWT2_E_DTYPE = -4,      /* unknown dtype, or dtype not valid for wavelet    */
    DWT2_E_WAVELET = -5,    /* unknown wavelet                                  */
    DWT2_E_BOUNDARY = -6,   /* unknown boundary extension                       */
    DWT2_E_PITCH = -7,      /* pitch < width                                    */
    DWT2_E_WORKSPACE = -8,  /* workspace NULL or smaller than required          */
    DWT2_E_ALIAS = -9,      /* src, dst or workspace overlap                    */
    DWT2_E_HIP = -10,       /* HIP runtime error at launch                      */
    DWT2_E_FLAGS = -11,     /* unknown flag, or flag not valid for the wavelet  */
    DWT2_E_COUNT = -12,     /* batched call: count < 1; plane batch: planes < 1 */
    DWT2_E_SCRATCH = -13,   /* dwt2_fwd_noalloc: the call needs more workspace
                               than DWT2_SCRATCH_BYTES                          */
    DWT2_E_TIMEOUT = -14    /* dwt2_workspace_status: a dependency wait of the
                               persistent forward ran out of time; the outputs
                               of that call are invalid                         */
} dwt2_status;

typedef enum {
    DWT2_CDF97 = 0,         /* CDF 9/7, float storage (F32, BF16, F16)          */
    DWT2_CDF53_REV = 1,     /* reversible integer CDF 5/3, I32 storage only     */
    DWT2_CDF53 = 2,         /* real-valued CDF 5/3 (the paper's 5/3, Section
                               "Evaluation"), float storage; p = -1/2,
                               u = 1/4, LL * 2, HH * 1/2 (zeta = sqrt(2))    */
    DWT2_DD137 = 3          /* Deslauriers-Dubuc 13/7 (Section "Evaluation"),
                               float storage: one pair of four-tap steps,
                               odd -= (9 (e[m] + e[m+1]) - (e[m-1] + e[m+2])) / 16,
                               even += (9 (o[m-1] + o[m]) - (o[m-2] + o[m+1])) / 32,
                               LL * 2, HH * 1/2 (zeta = sqrt(2)); borders
                               reflect the pixel position of each sample.
                               Forward / inverse on DWT2_ALGO_LDS kernel
                               configurations only (the default for it).   */
} dwt2_wavelet;

typedef enum {
    DWT2_F32 = 0,
    DWT2_BF16 = 1,
    DWT2_F16 = 2,
    DWT2_I32 = 3
} dwt2_dtype;

typedef enum {
    DWT2_SYMMETRIC_WHOLE = 0
} dwt2_boundary;

/* Flags (bitwise or). */
#define DWT2_FLAG_SPLIT 1u   /* P = P0 + P1, U = U0 + U1 operation-count reduction
                                (Section "Optimization Approach"); CDF 9/7 only.
                                Same values up to FP32 rounding; applied in tiles
                                away from the image border.                    */
#define DWT2_FLAG_SEPARABLE 2u  /* the comparison scheme of Section "Proposed
                                Schemes": every fused step replaced by its
                                horizontal and its vertical separable lifting
                                step, one work-group barrier each (8 barriers
                                per level for CDF 9/7, 4 for 5/3, against 4 and
                                2).  Same values up to FP32 rounding (5/3:
                                bit-identical).  dwt2_fwd / dwt2_inv (and their
                                _planes forms) with a DWT2_ALGO_TILE
                                configuration only; not with DWT2_FLAG_SPLIT. */
#define DWT2_FLAG_FACTORED 4u   /* the fused steps of Section "Proposed
                                Schemes" (one barrier each, as without the
                                flag), each evaluated as its horizontal then
                                its vertical factor in registers: a wave holds
                                whole tile rows, so the horizontal factor needs
                                no barrier, and the vertical factor reads the
                                neighbour's intermediate instead of recomputing
                                it.  8 operations per 2x2 block and fused step
                                instead of 11 (the split: 9).  Same values up
                                to FP32 rounding (5/3: bit-identical).  Same
                                restrictions as DWT2_FLAG_SEPARABLE; not
                                together with it.                            */
#define DWT2_FLAG_POLYCONV 8u   /* the non-separable polyconvolution scheme of
                                Section "Proposed Schemes": each pair of lifting
                                steps as one step N_{P,U} (V = P U + 1), every
                                output computed from the step's inputs over a
                                3 x 3 block neighbourhood, one barrier per pair
                                (2 per CDF 9/7 level).  CDF 9/7 only (the paper
                                gives it for wavelets of several pairs);
                                forward / inverse on DWT2_ALGO_LDS kernel
                                configurations (the default with this flag).
                                Same values up to FP32 rounding.             */
#define DWT2_FLAG_FUSED 32u  /* the fused steps T_P, S_U evaluated directly (the
                                paper's formulas).  Without any scheme flag the
                                fused steps run, evaluated directly for 4-byte
                                samples, and for BF16 / FP16 storage on
                                DWT2_ALGO_TILE configurations in the factored
                                form of DWT2_FLAG_FACTORED (same steps and
                                barriers, fewer operations: with half the bytes
                                per pixel that kernel is bound by its
                                arithmetic); this flag asks for the direct
                                evaluation everywhere.  Not together with
                                another scheme flag.                         */
#define DWT2_FLAG_PERSISTENT 16u  /* dwt2_fwd / dwt2_fwd_planes /
                                dwt2_fwd_batched: every level in one persistent
                                launch (after a planner launch) instead of one
                                launch per level; same values (bit-identical).
                                CDF 9/7, fused, split or factored steps,
                                DWT2_ALGO_TILE configurations, at most 65536 planes; not for
                                the inverse or adjoint (DWT2_E_FLAGS).  One
                                level is one launch either way.  See
                                dwt2_fwd_batched for its waits.              */
/* Kernel configuration: bits 8..15 hold 1 + the index of a configuration
 * listed by dwt2_kernel_config(); 0 selects the library default.  Every
 * configuration computes the same values (bit-identical for the same other
 * flags); they differ only in how the work is laid out on the GPU. */
#define DWT2_FLAG_KERNEL_SHIFT 8
#define DWT2_FLAG_KERNEL_MASK 0xff00u
#define DWT2_FLAG_KERNEL(i) (((unsigned)(i) + 1u) << DWT2_FLAG_KERNEL_SHIFT)
#define DWT2_NUM_KERNEL_CONFIGS 10

/* Kernel algorithms (dwt2_kernel_config). */
#define DWT2_ALGO_TILE 0     /* work-group tile in VGPRs, waves stacked
                                vertically, one LDS barrier per fused step */
#define DWT2_ALGO_STREAM 1   /* each wave64 walks down a column strip with a
                                register window; no LDS, no barrier */
#define DWT2_ALGO_LDS 2      /* the tile and its halo as the four polyphase
                                planes in LDS, one 2-D stencil and one barrier
                                per step (the paper's on-chip-memory design);
                                runs the fused, separable and polyconvolution
                                schemes of the float wavelets, forward and
                                inverse; CDF results bit-identical to the
                                DWT2_ALGO_TILE ones for the fused and
                                separable schemes */

/* One image of a batched call.  Pitches in elements. */
typedef struct {
    const void* src;
    void* dst;
    int32_t height;
    int32_t width;
    int64_t src_pitch;
    int64_t dst_pitch;
} dwt2_image;

/* Largest level count for which every transformed level is at least 2 x 2;
 * 0 if height or width < 2. */
int dwt2_max_levels(int32_t height, int32_t width);

/* Device workspace (bytes) that dwt2_fwd / dwt2_inv / dwt2_adj need for this
 * shape, level count and storage type (0 for one level): the intermediate LL
 * bands, and for the persistent forward also its work tables.  Returns a
 * dwt2_status. */
int dwt2_workspace_bytes(int32_t height, int32_t width, int levels,
                         dwt2_dtype dtype, size_t* bytes);

/* Forward transform (Section "Proposed Schemes", non-separable lifting):
 * src = image (height x width, src_pitch), dst = Mallat pyramid
 * (height x width, dst_pitch).  Multi-level: levels >= 1, one launch per
 * level (DWT2_FLAG_PERSISTENT: one persistent launch for all levels). */
int dwt2_fwd(const void* src, void* dst, int32_t height, int32_t width,
             int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
             dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
             unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream);

/* Inverse transform: src = Mallat pyramid (height x width, src_pitch), dst =
 * image (height x width, dst_pitch); arguments, workspace and errors as for
 * dwt2_fwd.  It inverts the factorisation of eq. (2) of Section "Background":
 * the lifting pairs in reverse order, each step with its coefficient negated.
 * With the fused steps of Section "Proposed Schemes" this is S_{-U} then
 * T_{-P} per pair: the horizontal and vertical factors of a fused step act on
 * different axes and commute, so the inverse of S_U is S_{-U} (its U U* term
 * keeps a + sign), and likewise for T_P.  The scaling is undone first.  For
 * the integer 5/3 the vertical half of each fused step is undone before the
 * horizontal half, which inverts it exactly. */
int dwt2_inv(const void* src, void* dst, int32_t height, int32_t width,
             int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
             dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
             unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream);

/* Adjoint (transpose) of dwt2_fwd: src = cotangent in Mallat layout, dst =
 * W^T src in image layout.  The transposed fused steps run in reverse order,
 * coarsest level first; at the borders the transposes of the symmetric
 * extension are used (they are not a symmetric extension).  CDF 9/7 only;
 * DWT2_FLAG_SPLIT is not accepted. */
int dwt2_adj(const void* src, void* dst, int32_t height, int32_t width,
             int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
             dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
             unsigned flags, void* workspace, size_t workspace_bytes,
             void* stream);

/* Plane batches (channels, batch items): `planes` images of the same shape
 * and pitch whose origins lie `src_plane_stride` / `dst_plane_stride`
 * elements apart, transformed as dwt2_fwd / dwt2_inv / dwt2_adj would
 * transform each one (bit-identical results), with one launch per level for
 * all planes.  planes >= 1 (else DWT2_E_COUNT); with planes > 1 each stride
 * must cover a whole plane, (height - 1) * pitch + width elements (else
 * DWT2_E_PITCH); no plane of src may overlap any of dst or the workspace.
 * The workspace holds the intermediate LL bands of every plane:
 * dwt2_workspace_bytes_planes, which returns a dwt2_status. */
int dwt2_workspace_bytes_planes(int32_t height, int32_t width, int levels, dwt2_dtype dtype,
                                int32_t planes, size_t* bytes);
int dwt2_fwd_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride,
                    int64_t dst_plane_stride, int32_t height, int32_t width, int64_t src_pitch,
                    int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
                    dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream);
int dwt2_inv_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride,
                    int64_t dst_plane_stride, int32_t height, int32_t width, int64_t src_pitch,
                    int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
                    dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream);
int dwt2_adj_planes(const void* src, void* dst, int32_t planes, int64_t src_plane_stride,
                    int64_t dst_plane_stride, int32_t height, int32_t width, int64_t src_pitch,
                    int64_t dst_pitch, dwt2_dtype dtype, dwt2_wavelet wavelet, int levels,
                    dwt2_boundary boundary, unsigned flags, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Describe kernel configuration `index` (0 .. DWT2_NUM_KERNEL_CONFIGS-1):
 * algorithm (DWT2_ALGO_*), wave64s per work-group, block rows per lane
 * (tile) or rows of loads in flight (stream), and the output size one
 * work-group tile (or one wave segment) covers in 2x2-pixel blocks: core_cols
 * columns by core_rows rows.  Any output pointer may be NULL.  Returns
 * DWT2_OK or DWT2_E_FLAGS for an unknown index. */
int dwt2_kernel_config(int index, int* algorithm, int* waves, int* rows, int* core_cols, int* core_rows);

/* Device workspace (bytes) for dwt2_fwd_batched on these images, with or
 * without DWT2_FLAG_PERSISTENT: the work tables and every image's
 * intermediate LL bands.  `images` is a host array.  Returns a dwt2_status. */
int dwt2_workspace_bytes_batched(const dwt2_image* images, int count, dwt2_dtype dtype, int levels,
                                 size_t* bytes);

/* Batched forward CDF 9/7 (Section "Proposed Schemes", non-separable lifting,
 * applied to each image as dwt2_fwd would): `count` independent images of any
 * (uneven) sizes, every one transformed to `levels` levels, on `stream`.  By
 * default a planner launch plus one launch per level, the launch of a level
 * covering the tiles of all images.  With DWT2_FLAG_PERSISTENT: a planner
 * launch plus one persistent launch for every level; its work-groups take
 * tiles (of every image) from work queues, level after level, and a tile of
 * level l >= 1 first waits until the tiles of level l - 1 whose LL rows it
 * reads have finished, so the levels overlap.  Such a wait is bounded
 * (200 ms; the environment variable DWT2_WAIT_LIMIT_US, read at each call,
 * sets another limit): if one runs out the call still ends, with its outputs
 * invalid and an error word set in the workspace (dwt2_workspace_status).
 * The images are given twice with identical contents: `host_images` (host
 * memory, used for the argument checks and the grid sizes) and
 * `device_images` (device memory, read by the kernels; it must stay valid
 * until the launches have run).  The call performs no copies or allocations
 * and can be captured in a graph.  Float storage (F32, BF16, F16); flags:
 * DWT2_FLAG_SPLIT, DWT2_FLAG_PERSISTENT and a tile kernel configuration (any
 * DWT2_ALGO_TILE index of dwt2_kernel_config).  No image's src or dst may
 * overlap the workspace, and no image's dst may overlap the dst or the src of
 * any image (sources may overlap one another): every such batch is rejected
 * with DWT2_E_ALIAS.  The sum over the images of one level's tiles must stay
 * below 2^31 - 2^16 (else DWT2_E_SHAPE).  Results equal dwt2_fwd on each
 * image (bit-identical for the same configuration). */
int dwt2_fwd_batched(const dwt2_image* host_images, const dwt2_image* device_images, int count,
                     dwt2_dtype dtype, dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
                     unsigned flags, void* workspace, size_t workspace_bytes, void* stream);

/* Outcome of the last persistent forward (DWT2_FLAG_PERSISTENT) that used a
 * workspace: `header` is a host copy of the first DWT2_WORKSPACE_STATUS_BYTES
 * bytes of that workspace, taken after the call has run.  Returns DWT2_OK, or
 * DWT2_E_TIMEOUT if a dependency wait ran out of time (outputs invalid). */
#define DWT2_WORKSPACE_STATUS_BYTES 4
int dwt2_workspace_status(const void* header);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): dwt2_fwd with
 * no workspace argument.  The intermediate LL bands go to a fixed device
 * array of DWT2_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (enough for any level count of an 8192 x 8192 FP32
 * image); the call allocates and frees nothing.  Arguments, results and
 * errors as dwt2_fwd (bit-identical results); a call that needs more
 * workspace than the array (dwt2_workspace_bytes) returns DWT2_E_SCRATCH
 * before any HIP call.  The first call on a device looks up the array's
 * address there (current device).  All calls on one GPU share its array;
 * what must start at zero there (the persistent path's counters) is cleared
 * by each call's own planner launch: calls ordered on one stream are safe,
 * calls that can overlap in time on one GPU (other streams, other host
 * threads) race on it. */
#define DWT2_SCRATCH_BYTES ((size_t)96 << 20)
int dwt2_fwd_noalloc(const void* src, void* dst, int32_t height, int32_t width,
                     int64_t src_pitch, int64_t dst_pitch, dwt2_dtype dtype,
                     dwt2_wavelet wavelet, int levels, dwt2_boundary boundary,
                     unsigned flags, void* stream);

/* Text of a dwt2_status. */
const char* dwt2_status_string(int status);

/* Text of the last HIP error reported as DWT2_E_HIP on this thread. */
const char* dwt2_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DWT2_H */
