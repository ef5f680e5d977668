/*
 * icl.h - C ABI of the MI355X (gfx950) stencil image library.
 *
 * The library implements the per-pixel neighbourhood kernels that the ImageCL
 * paper (Falch & Elster, arXiv 1605.06399) generates and auto-tunes: a kernel is
 * the work of one logical thread per pixel of an Image grid, reading a bounded
 * neighbourhood with a boundary condition (Section 5), launched from a
 * standalone host function (Section 5.1).  Each entry point below is such a host
 * function for one stencil; the variant it launches (work-group shape, pixels
 * per thread, LDS staging or direct loads, unrolling: the Table 1 parameters)
 * is chosen per device by the library's auto-tuner (Section 4), or forced.
 *
 * Conventions shared by every entry point
 *  - Images are 2-D, row-major, x (the paper's idx) fastest.  Pixel (x, y) of an
 *    image lives at  base + y * pitch + x * elem_size ; pitches are in BYTES and
 *    must satisfy pitch >= width * elem_size and pitch % elem_size == 0.
 *  - Boundary: clamped (Section 5, Fig. 3a): a read outside the image returns
 *    the closest pixel inside, i.e. x -> min(max(x, 0), width-1), same for y.
 *    The convolution calls with an icl_border argument also take the constant
 *    condition (Fig. 3b): every read outside the image returns a given constant.
 *  - Image, tap and workspace pointers are DEVICE pointers unless stated.
 *    Filter taps are float32 in device memory and are read at run time, so taps
 *    updated in place are seen by later calls and by graph replays.
 *  - Correlation orientation: tap index k = (j+r)*(2r+1) + (i+r) multiplies the
 *    input at offset (x+i, y+j); no flip.
 *  - The caller owns every buffer.  Hot calls allocate nothing and never
 *    synchronise; they enqueue on `stream` (a hipStream_t; NULL = the null
 *    stream) and return.  Scratch memory is passed in as `workspace`, sized by
 *    icl_workspace_size().
 *  - Input and output images must not overlap (ICL_ERR_ALIAS): the paper's
 *    language forbids aliasing and local-memory staging needs read-only inputs
 *    (Section 5.2, memory spaces).
 *  - Arithmetic is float32 with float32 accumulation (unless the caller opts into
 *    ICL_MATH_F16_SPLIT, see icl_set_math); float16 / bfloat16 storage is decoded
 *    exactly on load and rounded to nearest even on store.
 *  - width == 0 or height == 0 is an empty image: the call returns ICL_OK and
 *    touches nothing.  Negative sizes are ICL_ERR_INVALID_VALUE.
 *  - Errors: arguments are checked on the host before anything is launched and
 *    an icl_status is returned; no call aborts or throws.  A failing HIP call
 *    returns ICL_ERR_HIP and its hipError_t is kept per thread
 *    (icl_last_hip_error()).
 */
#ifndef ICL_H
#define ICL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum icl_status {
    ICL_OK = 0,
    ICL_ERR_INVALID_VALUE = 1, /* null pointer, negative size, bad count or enum */
    ICL_ERR_PITCH = 2,         /* pitch < width * elem or not a multiple of elem */
    ICL_ERR_RADIUS = 3,        /* radius outside the supported range */
    ICL_ERR_DTYPE = 4,         /* storage type not supported by this entry point */
    ICL_ERR_ALIAS = 5,         /* an output overlaps an input */
    ICL_ERR_WORKSPACE = 6,     /* workspace missing or smaller than icl_workspace_size() */
    ICL_ERR_NO_DEVICE = 7,     /* no HIP device visible */
    ICL_ERR_HIP = 8,           /* a HIP runtime call failed (see icl_last_hip_error) */
    ICL_ERR_UNSUPPORTED = 9,   /* valid request the library does not implement */
    ICL_ERR_TUNE_CACHE = 10    /* tune cache unreadable or written for another device */
} icl_status;

/* pixel storage types; ICL_U8 (unsigned char) only for icl_conv2d_u8 */
typedef enum icl_dtype { ICL_F32 = 0, ICL_F16 = 1, ICL_BF16 = 2, ICL_U8 = 3 } icl_dtype;

/* boundary conditions (Section 5, Fig. 3) */
typedef enum icl_border {
    ICL_BORDER_CLAMP = 0,     /* a read outside returns the closest pixel inside */
    ICL_BORDER_CONSTANT = 1   /* a read outside returns the given constant */
} icl_border;

/* operations, for icl_workspace_size / icl_tune / variant control */
typedef enum icl_op {
    ICL_OP_CONV_SEP = 0,
    ICL_OP_CONV2D = 1,
    ICL_OP_HARRIS = 2,
    ICL_OP_NMS = 3,
    ICL_OP_CONV_SEP_BATCHED = 4,
    ICL_OP_BANK_FWD = 5,
    ICL_OP_BANK_BWD_INPUT = 6,
    ICL_OP_BANK_BWD_FILTER = 7,
    ICL_OP_SSE_LOSS = 8,
    ICL_OP_BANK_FWD_SSE = 9,
    ICL_OP_CONV2D_U8 = 10,
    ICL_OP_CORNERS = 11,
    ICL_OP_CONV3D_SEP = 12,
    ICL_OP_COUNT = 13
} icl_op;

#define ICL_MAX_RADIUS 16          /* largest stencil radius accepted by the convolution calls */
#define ICL_MAX_WINDOW_RADIUS 7    /* largest Harris window radius */
#define ICL_MAX_NMS_RADIUS 7
#define ICL_MAX_U8_RADIUS 7        /* largest radius of icl_conv2d_u8 (keeps its int32 sum exact) */
#define ICL_MAX_U8_SHIFT 16
#define ICL_MAX_RADIUS_3D 7        /* largest radius of icl_conv3d_sep */

/* ------------------------------------------------------------------ library */

/* Initialise the runtime side (device query, tune cache).  Optional: every call
 * initialises lazily.  Returns ICL_ERR_NO_DEVICE when no GPU is visible. */
icl_status icl_init(void);

const char* icl_status_string(icl_status s);   /* static string, never NULL */
int icl_last_hip_error(void);                   /* hipError_t of this thread's last failing HIP call */
const char* icl_version(void);

/* Scratch bytes an operation needs for the given problem (0 when none).  For
 * ICL_OP_CONV_SEP this is the float32 row-pass intermediate of the two-pass
 * variants; for ICL_OP_HARRIS the two float32 gradient images of the split
 * (Sobel kernel + Harris kernel) variant; for ICL_OP_BANK_BWD_FILTER,
 * ICL_OP_SSE_LOSS and ICL_OP_BANK_FWD_SSE the per-block partial sums; for ICL_OP_CORNERS the
 * two-kernel variant's float32 response image and, for window radii above 3, the gradient
 * images (`radius` is the window radius); for ICL_OP_CONV3D_SEP the two float32 intermediate
 * volumes of the three-pass variant (`n` is the depth).  Callers that always pass this
 * much workspace may use every variant.  `n` and `f` are the batch and filter
 * counts of the filter-bank ops, `n` the depth for ICL_OP_CONV3D_SEP (ignored otherwise). */
icl_status icl_workspace_size(icl_op op, int width, int height, int n, int f, int radius,
                              icl_dtype dtype, size_t* bytes /* host */);

/* ------------------------------------------------------------------ separable convolution
 * Paper: Section 6, separable convolution benchmark (row kernel R and column
 * kernel C, Table 2); the discussion names fusing the two passes with the
 * intermediate in local memory as the optimisation ImageCL could not express.
 *   T(x,y) = sum_{i=-r..r} taps_x[i+r] * src(x+i, y)
 *   dst(x,y) = sum_{j=-r..r} taps_y[j+r] * T(x, y+j)        (reads clamped)
 * T is kept in float32 (never rounded to the storage type).
 *   src, dst      : device images of `dtype`, pitches in bytes
 *   taps_x/taps_y : device float32 arrays of 2r+1 taps, r in [0, ICL_MAX_RADIUS]
 *   workspace     : device scratch of icl_workspace_size(ICL_OP_CONV_SEP) bytes, or
 *                   NULL / too small: then only the fused single-pass variants run
 *                   (ICL_ERR_WORKSPACE if a two-pass variant is forced). */
icl_status icl_conv_sep(const void* src, size_t src_pitch, void* dst, size_t dst_pitch,
                        int width, int height, icl_dtype dtype,
                        const float* taps_x, const float* taps_y, int radius,
                        void* workspace, size_t workspace_bytes, void* stream);

/* icl_conv_sep under a chosen boundary condition (Section 5, Fig. 3; the paper's
 * separable benchmark uses the constant one).  With ICL_BORDER_CONSTANT the filter
 * is the 2-D correlation with taps taps_y (x) taps_x of the image extended by
 * `constant`: a row of T outside the image is sum_i taps_x[i] * constant (summed
 * in tap order), not the constant itself.  With ICL_BORDER_CLAMP (`constant`
 * ignored) this is exactly icl_conv_sep.  ICL_ERR_INVALID_VALUE for another
 * `border`; every other argument as in icl_conv_sep. */
icl_status icl_conv_sep_border(const void* src, size_t src_pitch, void* dst, size_t dst_pitch,
                               int width, int height, icl_dtype dtype,
                               const float* taps_x, const float* taps_y, int radius,
                               icl_border border, float constant,
                               void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ 2-D correlation
 * Paper: Section 6, non-separable convolution benchmark (Table 3): a full
 * (2r+1)^2 filter whose taps are known only at run time.
 *   dst(x,y) = sum_{j,i=-r..r} taps[(j+r)(2r+1) + (i+r)] * src(x+i, y+j)
 *   taps : device float32, (2r+1)^2 values, row (j) major. */
icl_status icl_conv2d(const void* src, size_t src_pitch, void* dst, size_t dst_pitch,
                      int width, int height, icl_dtype dtype,
                      const float* taps, int radius, void* stream);

/* icl_conv2d under a chosen boundary condition: with ICL_BORDER_CONSTANT every
 * read outside the image is `constant` (Section 5, Fig. 3b).  With
 * ICL_BORDER_CLAMP (`constant` ignored) this is exactly icl_conv2d. */
icl_status icl_conv2d_border(const void* src, size_t src_pitch, void* dst, size_t dst_pitch,
                             int width, int height, icl_dtype dtype,
                             const float* taps, int radius, icl_border border, float constant,
                             void* stream);

/* ------------------------------------------------------------------ 3-D separable correlation
 * Paper: Section 5, the Image type's 3-D indexing; the separable passes of the Section 6
 * benchmark with a third (z) pass.  A volume is `depth` slices of `height` rows:
 * voxel (x, y, z) lives at base + z * slice_pitch + y * row_pitch + x * elem_size.
 *   T1(x,y,z) = sum_i taps_x[i+r] V(x+i, y, z)
 *   T2(x,y,z) = sum_j taps_y[j+r] T1(x, y+j, z)
 *   dst(x,y,z) = sum_k taps_z[k+r] T2(x, y, z+k)
 * i.e. the 3-D correlation with taps taps_z (x) taps_y (x) taps_x of the volume extended by
 * the boundary condition (clamp per axis, or `constant` for every voxel outside; with the
 * constant the intermediates outside are the passes of the constant, as for icl_conv_sep_border).
 * Intermediates are float32.
 *   row_pitch  >= width * elem, slice_pitch >= (height-1) * row_pitch + width * elem, both
 *              multiples of elem (ICL_ERR_PITCH)
 *   radius     : 0 .. ICL_MAX_RADIUS_3D (the single-pass variants cover 0..3)
 *   workspace  : icl_workspace_size(ICL_OP_CONV3D_SEP, width, height, depth) bytes for the
 *                three-pass variant, or NULL (then radii above 3 are ICL_ERR_WORKSPACE). */
icl_status icl_conv3d_sep(const void* src, size_t src_row_pitch, size_t src_slice_pitch,
                          void* dst, size_t dst_row_pitch, size_t dst_slice_pitch,
                          int width, int height, int depth, icl_dtype dtype,
                          const float* taps_x, const float* taps_y, const float* taps_z, int radius,
                          icl_border border, float constant,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ 8-bit 2-D correlation
 * Paper: Section 6, non-separable convolution benchmark, run on unsigned char
 * pixels with a 5x5 filter known at run time and the clamped boundary.  Integer
 * arithmetic, exact:
 *   S(x,y)   = sum_{j,i=-r..r} taps[(j+r)(2r+1) + (i+r)] * src(x+i, y+j)
 *   dst(x,y) = min(max((S + b) >> shift, 0), 255),  b = 2^(shift-1), or 0 if shift = 0
 * (>> is the arithmetic shift, i.e. floor division: round to nearest, ties up,
 * then saturate).  The sum is exact in 32-bit integers for every input.
 *   src, dst : device unsigned char images, pitches in bytes (any alignment)
 *   taps     : device int16, (2r+1)^2 values, row (j) major; r in [0, ICL_MAX_U8_RADIUS]
 *   shift    : 0 .. ICL_MAX_U8_SHIFT, else ICL_ERR_INVALID_VALUE
 *   border   : ICL_BORDER_CLAMP, or ICL_BORDER_CONSTANT with `constant` in 0..255
 *              (the value of every read outside the image; else ICL_ERR_INVALID_VALUE).
 * Every variant returns the same bytes. */
icl_status icl_conv2d_u8(const uint8_t* src, size_t src_pitch, uint8_t* dst, size_t dst_pitch,
                         int width, int height, const int16_t* taps, int radius, int shift,
                         icl_border border, int constant, void* stream);

/* ------------------------------------------------------------------ Harris corner response
 * Paper: Section 6, Harris corner detection, run there as a Sobel kernel
 * (Table 4) followed by a Harris kernel that reads the gradient images dx, dy as
 * Images (Table 5), so the window's reads are clamped on the gradient images.
 *   Ix = sum s[j] d[i] src(x+i,y+j),  Iy = sum d[j] s[i] src(x+i,y+j),
 *        s = (1,2,1), d = (-1,0,1)      (unnormalised Sobel)
 *   Sxx = sum_{j,i} g[j] g[i] Ix^2(x+i, y+j), Syy likewise with Iy^2, Sxy with Ix*Iy
 *   resp = Sxx*Syy - Sxy^2 - k*(Sxx+Syy)^2
 *   src, resp    : float32 device images
 *   window_taps  : device float32, 2*window_radius+1 taps g (window = outer product g g^T),
 *                  window_radius in [0, ICL_MAX_WINDOW_RADIUS]
 *   workspace    : icl_workspace_size(ICL_OP_HARRIS) bytes for the split variant, or NULL. */
icl_status icl_harris(const float* src, size_t src_pitch, float* resp, size_t resp_pitch,
                      int width, int height, const float* window_taps, int window_radius,
                      float k, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ non-maximum suppression
 * Final stage of corner detection (not defined in the paper; it thresholds the
 * Harris response to a corner mask).
 *   mask(x,y) = 1 if resp(x,y) > threshold and resp(x,y) >= resp(x+i,y+j) for all
 *               |i|,|j| <= radius (reads clamped, so outside neighbours are ignored),
 *               else 0.
 *   resp : float32 device image;  mask : uint8 device image (pitch in bytes);
 *   radius in [1, ICL_MAX_NMS_RADIUS]. */
icl_status icl_nms(const float* resp, size_t resp_pitch, uint8_t* mask, size_t mask_pitch,
                   int width, int height, int radius, float threshold, void* stream);

/* ------------------------------------------------------------------ corner detection, fused
 * Paper: Section 6, Harris corner detection (a Sobel kernel and a Harris kernel, Tables 4
 * and 5); the discussion names fusing such stages as what the language could not express.
 * This call is icl_harris followed by icl_nms in one pass: the response R (exactly the
 * float32 expression of icl_harris) stays in registers, and
 *   mask(x,y) = 1 iff R(x,y) > threshold and R(x,y) >= R at every pixel of the
 *               (2 nms_radius + 1)^2 window (reads of R clamped), else 0.
 * HBM traffic 5 B/px (image in, mask out) instead of 13 B/px for the two calls.
 *   src          : device float32 image; window_taps, window_radius, k as in icl_harris
 *   mask         : device uint8 image (any pitch)
 *   nms_radius   : 1 .. ICL_MAX_NMS_RADIUS (the single-pass variants cover radius 1 and
 *                  window radius <= 3; other radii run the two kernels)
 *   resp         : optional device float32 image (NULL: the response is not written);
 *                  with it the response is also written, in one pass
 *   workspace    : icl_workspace_size(ICL_OP_CORNERS, ..., radius = window_radius) bytes,
 *                  needed only when the two-kernel variant runs (NMS radius > 1 or window
 *                  radius > 3): room for the response when resp is NULL, plus the gradient
 *                  images for window radii above 3 (else ICL_ERR_WORKSPACE).
 * No output may overlap the image or each other (ICL_ERR_ALIAS). */
icl_status icl_corners(const float* src, size_t src_pitch, uint8_t* mask, size_t mask_pitch,
                       int width, int height, const float* window_taps, int window_radius, float k,
                       int nms_radius, float threshold, float* resp, size_t resp_pitch,
                       void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ batched separable convolution
 * Many images of uneven size, each with its own radius and taps, in ONE
 * persistent kernel launch (work is a table of tiles, each naming its image).
 * Same arithmetic as icl_conv_sep, per image, fused single pass. */
typedef struct icl_image_desc {
    const void* src;       /* device */
    void* dst;             /* device */
    size_t src_pitch;      /* bytes */
    size_t dst_pitch;      /* bytes */
    int width, height;
    int radius;            /* 0 .. 7 */
    const float* taps_x;   /* device, 2r+1 */
    const float* taps_y;   /* device, 2r+1 */
} icl_image_desc;

typedef struct icl_batch_plan icl_batch_plan;   /* opaque */

/* Validates every descriptor (host array of `count`), builds the tile table and
 * uploads it (this call allocates device memory and synchronises; it is not
 * capture-safe).  All images share `dtype`. */
icl_status icl_batch_plan_create(const icl_image_desc* descs, int count, icl_dtype dtype,
                                 icl_batch_plan** plan /* host out */);
/* The auto-tuner for a plan (the paper's Section 4 search, per device): runs each walk of
 * the plan (tile shapes and orders, the strip walk) on the plan's own buffers, rejects a
 * walk whose output differs from the default walk's, times the rest with HIP events and
 * keeps the fastest for this plan; later icl_conv_sep_batched calls (and graphs created
 * after it) launch that walk.  It writes the plan's outputs, allocates, synchronises and
 * must not be called during stream capture.  A forced variant still takes precedence. */
icl_status icl_batch_plan_tune(icl_batch_plan* plan, void* stream);
/* Variant (walk) index icl_conv_sep_batched would launch for this plan (host out). */
icl_status icl_batch_plan_variant(const icl_batch_plan* plan, int* index);
/* One persistent launch over the plan's tiles.  Allocates nothing: capture-safe. */
icl_status icl_conv_sep_batched(const icl_batch_plan* plan, void* stream);
/* Number of tiles and total pixels of a plan (host out pointers, either may be NULL). */
icl_status icl_batch_plan_info(const icl_batch_plan* plan, long long* tiles, long long* pixels);
void icl_batch_plan_destroy(icl_batch_plan* plan);

/* Capture icl_conv_sep_batched(plan) into a HIP graph and instantiate it.  The
 * graph holds one kernel node; replaying it re-reads images and taps, so new
 * data in the same buffers is picked up.  `*exec` is a hipGraphExec_t. */
icl_status icl_batch_graph_create(const icl_batch_plan* plan, void** exec /* host out */);
icl_status icl_graph_launch(void* exec, void* stream);
void icl_graph_destroy(void* exec);

/* ------------------------------------------------------------------ differentiable filter bank
 * F learnable filters of radius r applied to N single-channel images (clamped
 * correlation), with the adjoint kernels for backpropagation.  Dense NCHW
 * float32 tensors, element offsets 64-bit:
 *   x  [n][h][wd]   w [f][2r+1][2r+1]   y, gy [n][f][h][wd]   gx [n][h][wd]
 *   forward      y[n,f,p]  = sum_k w[f,k] x[n, clamp(p+k)]
 *   input grad   gx[n,q]   = sum over (f, p, k) with clamp(p+k) = q of w[f,k] gy[n,f,p]
 *   filter grad  gw[f,k]   = sum_{n,p} gy[n,f,p] x[n, clamp(p+k)]   (fixed-order reduction)
 * radius in [1, 4] and f in [1, 64]. */
icl_status icl_bank_fwd(const float* x, const float* w, float* y, int n, int f, int h, int wd,
                        int radius, void* stream);
/* The adjoints take an optional `scale` (device float32 scalar, NULL = 1) multiplying their
 * output: the chain-rule factor of an upstream gradient dJ/dL on a scalar loss L, so that
 * gx = scale * dL/dx and gw = scale * dL/dw come out of the kernels with no extra pass. */
icl_status icl_bank_bwd_input(const float* gy, const float* w, float* gx, int n, int f, int h, int wd,
                              int radius, const float* scale, void* stream);
icl_status icl_bank_bwd_filter(const float* gy, const float* x, float* gw, int n, int f, int h, int wd,
                               int radius, const float* scale, void* workspace, size_t workspace_bytes,
                               void* stream);

/* Sum-of-squares loss L = sum (y - t)^2 over `count` elements and its gradient
 * gy = 2 (y - t) (gy may be NULL).  `loss` is a device float32 written with L;
 * the reduction order is fixed, so results are reproducible run to run. */
icl_status icl_sse_loss(const float* y, const float* t, float* gy, long long count, float* loss,
                        void* workspace, size_t workspace_bytes, void* stream);

/* The filter-bank forward fused with the sum-of-squares loss against a target
 * t [n][f][h][wd] (dense, float32):
 *   L = sum (y - t)^2 written to the device float32 `loss`, gy = 2 (y - t) written
 *   when gy != NULL, the forward output y written when y != NULL.
 * The training step of a learnable filter bank needs gy and L but not y, so with
 * y == NULL the 4-byte-per-element write of y and its re-read by the loss drop out.
 * y and gy are bit-identical to icl_bank_fwd followed by icl_sse_loss when both run
 * variants of one family: the FMA variants all sum the taps in one order, the matrix-core
 * (MFMA) variants in another (their results differ in rounding only).  L is accumulated in float64 per
 * work-group and summed in a fixed order, so it is reproducible run to run.
 *   workspace : icl_workspace_size(ICL_OP_BANK_FWD_SSE) bytes of device scratch
 *               (ICL_ERR_WORKSPACE if NULL or smaller).
 * Shapes, radius and filter limits as icl_bank_fwd; t, y, gy must not overlap x, w or
 * each other (ICL_ERR_ALIAS). */
icl_status icl_bank_fwd_sse(const float* x, const float* w, const float* t, float* y, float* gy, float* loss,
                            int n, int f, int h, int wd, int radius, void* workspace, size_t workspace_bytes,
                            void* stream);

/* icl_bank_fwd_sse without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no hipMalloc, hipFree or allocating routine, and never starts a
 * tuner search (a tune-cache miss takes the default variant).  The loss partials live in
 * a fixed device array of FWD_SSE_PARTS (2048) float64 values = 16 KiB, one copy per
 * device, looked up on the first call on that device (or by icl_init) and held until the
 * process ends.  The partial count is capped at that size for every problem, so no
 * problem size is rejected for lack of scratch.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (concurrent streams, threads)
 * race on it and must be serialised by the caller.  Each call writes every partial it
 * reads, so nothing needs clearing between calls.
 * Arguments, outputs, limits and errors as icl_bank_fwd_sse; y, gy and L are bit-identical
 * to icl_bank_fwd_sse's when both run the same variant. */
icl_status icl_bank_fwd_sse_noalloc(const float* x, const float* w, const float* t, float* y, float* gy,
                                    float* loss, int n, int f, int h, int wd, int radius, void* stream);

/* ------------------------------------------------------------------ auto-tuning and variants
 * The tuner plays the role of the paper's auto-tuner (Section 4 and the
 * discussion of tuning cost): it runs every precompiled candidate variant of an
 * operation on synthetic data of the given shape, rejects candidates whose
 * output differs from the plain variant's (byte for byte for ICL_OP_CONV2D_U8,
 * whose dtype is ICL_U8), times the rest with HIP events on
 * rotating buffers, and records the fastest in a per-device cache keyed by
 * (device, op, dtype, radius, size class).  Candidates are compiled ahead of
 * time, so a search costs only run time.
 * icl_tune allocates, synchronises and must not be called during stream capture. */
icl_status icl_tune(icl_op op, icl_dtype dtype, int radius, int width, int height, void* stream);

/* A problem for tuning and selection when more than the image size matters:
 *   depth : slices of a volume (ICL_OP_CONV3D_SEP)
 *   n, f  : batch and filter counts of the filter-bank ops (ICL_OP_BANK_*); width and
 *           height are then the image width and height
 * Unused fields are 0 or 1.  The cache keys on (op, dtype, radius, floor(log2(width *
 * height * depth * n)), f, icl_get_math()), so the later calls of the same problem class
 * pick the tuned variant.  icl_tune(op, ...) is icl_tune_problem with depth = n = f = 1.
 * ICL_ERR_INVALID_VALUE for a null pointer or sizes below 1; ranges as the operation's. */
typedef struct icl_problem {
    icl_op op;
    icl_dtype dtype;
    int radius;
    int width, height;
    int depth, n, f;
} icl_problem;
icl_status icl_tune_problem(const icl_problem* problem, void* stream);
/* Variant the next call of this problem would launch (host out). */
icl_status icl_selected_variant_problem(const icl_problem* problem, int* index);
/* Persist / reload the cache (JSON).  path NULL = $ICL_TUNE_CACHE or ~/.cache/icl/tune.json. */
/* The paper's model-guided search (Section 4) over the same candidates: time `samples`
 * randomly chosen candidates (seeded), fit a small neural-network model of log execution
 * time over the candidates' parameters (icl_perf_model_fit_predict), predict the rest, time
 * the `top_k` best-predicted, and cache the fastest measured.  With fewer than
 * samples + top_k + 1 candidates every candidate is timed.  `timed` (host, may be NULL)
 * receives the number of candidates timed.  samples >= 2, top_k >= 1, else
 * ICL_ERR_INVALID_VALUE; otherwise as icl_tune. */
icl_status icl_tune_model(icl_op op, icl_dtype dtype, int radius, int width, int height, int samples, int top_k,
                          unsigned long long seed, int* timed, void* stream);

/* The tuner's time model, exposed for inspection and testing (host memory, no device use):
 * fit a network with one hidden layer of `hidden` tanh units (inputs and target
 * standardised; full-batch Adam, `iters` steps, weights from a SplitMix64 stream of `seed`,
 * so the fit is deterministic) to the n rows of X [n][d] and targets y [n], then write its
 * predictions for the nq rows of Xq [nq][d] to yq.  ICL_ERR_INVALID_VALUE for null pointers,
 * n < 2, d < 1, hidden outside 1..256 or iters outside 1..10^6. */
icl_status icl_perf_model_fit_predict(const double* X, const double* y, int n, int d, const double* Xq, int nq,
                                      double* yq, int hidden, int iters, unsigned long long seed);

/* Arithmetic of the variants that tuning and default selection may pick.
 *   ICL_MATH_F32 (the default): only variants with float32 products and float32
 *     accumulation (vector FMA or the float32 matrix instructions), so every
 *     result meets the float32 error model of the conventions above.
 *   ICL_MATH_F16_SPLIT: also the matrix-core 2-D correlation ("mfma_f16x3") that
 *     splits each float32 operand into float16 hi + lo parts and adds three
 *     float16 products with float32 accumulation.  Besides float32 rounding its
 *     result errs by up to 2^-37 (2r+1)^2 M max|w| per pixel, M the largest |src|
 *     of the 64x64 tile holding the pixel: windows far darker than their tile's
 *     brightest pixel (about 2^20 below it) keep fewer bits than float32.  A
 *     caller opts in when its images have no such contrast.
 * The mode is process-wide.  Tune-cache entries are keyed by it, so a variant tuned
 * under one mode is never selected under the other; a forced variant
 * (icl_force_variant) runs whatever the mode.  ICL_ERR_INVALID_VALUE for another
 * value.  Not thread-safe against calls running concurrently on other threads. */
typedef enum icl_math { ICL_MATH_F32 = 0, ICL_MATH_F16_SPLIT = 1 } icl_math;
icl_status icl_set_math(icl_math mode);
icl_math icl_get_math(void);
/* Arithmetic a variant computes in (static string, NULL if out of range):
 *   "fp32_valu"   float32 vector FMA          "fp32_mfma"  float32 matrix instructions
 *   "fp16x3_mfma" float16 hi/lo split on the matrix cores (see ICL_MATH_F16_SPLIT)
 *   "int32_valu"  exact integer arithmetic (icl_conv2d_u8) */
const char* icl_variant_arith(icl_op op, int index);

icl_status icl_tune_save(const char* path);
icl_status icl_tune_load(const char* path);
void icl_tune_clear(void);

/* Environment (read once, at the first call that selects a variant):
 *   ICL_TUNE=off     ignore the tune cache: every call runs the forced or default variant
 *   ICL_TUNE=cache   (default) use tuned entries when present, the default otherwise
 *   ICL_TUNE=search  as cache, and on a miss tune that problem first (icl_tune, which
 *                    allocates and synchronises; skipped while the stream is capturing),
 *                    then save the cache, so an interrupted series of searches resumes
 *   ICL_TUNE_CACHE   cache file, loaded at that first call when it exists
 *   ICL_FORCE_VARIANT=op=index[,op=index...]   as icl_force_variant, e.g. "conv2d=3" */

/* Variant table of an operation (index 0 is always the plain one-pixel-per-thread kernel). */
int icl_variant_count(icl_op op);
const char* icl_variant_name(icl_op op, int index);     /* NULL if out of range */
/* Force a variant for every later call of `op` (-1 = back to tuned/default
 * selection); the analogue of the paper's directives that force optimisations
 * on or off.  A forced variant that cannot run a call (radius not compiled,
 * missing workspace) makes that call return ICL_ERR_UNSUPPORTED / ICL_ERR_WORKSPACE. */
icl_status icl_force_variant(icl_op op, int index);
/* Variant the next call with these parameters would launch (host out). */
icl_status icl_selected_variant(icl_op op, icl_dtype dtype, int radius, int width, int height,
                                int* index);

#ifdef __cplusplus
}
#endif

#endif /* ICL_H */
