/*
 * CPU oracle for the ImageCL stencil hot path (Falch & Elster, arXiv 1605.06399).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code with the HIP kernels.
 *
 * Every function is the plain definition of what the method computes, written
 * as straight loops in IEEE double precision (inputs are promoted from their
 * stored type, taps from float32).  Rows may be split across OpenMP threads;
 * that never changes the order of any sum.
 *
 * Pixel addressing follows the paper's Image type (Section 5): an image is
 * flattened row-major, the first index idx is x (fast), the second idy is y.
 * Boundary handling is the clamped condition of Section 5 / Fig. 3(a): a read
 * outside the image returns the closest pixel inside it.  Per axis that is
 * min(max(i, 0), n-1), and the per-axis clamp is the closest pixel in the
 * Euclidean sense too (corners included).  The convolutions also take the
 * constant condition of Fig. 3(b): a read outside the image returns a constant.
 *
 * Parity pins (all checked by the CPU test-suite, none by re-typing a formula):
 *   conv2d / conv_sep : delta filter reproduces the input bit-exactly; a shifted
 *                       delta reproduces the shifted image with closest-pixel
 *                       semantics found by brute-force distance search; a
 *                       constant image under taps summing to 1 stays constant;
 *                       the separable pair equals the brute-force outer-product
 *                       2-D filter; 1x1 images give X * sum(w); the 3x3 box
 *                       filter of Listing 1 on integer images is exact;
 *                       linearity and transposition.  Constant boundary: equal
 *                       to a correlation of the constant-padded image computed
 *                       by numpy slicing; hand-worked 3x3 box sums; a constant
 *                       image equal to the constant gives c * sum(w).
 *   conv3d_sep        : correlation of the padded volume by numpy slicing with
 *                       the outer-product taps (clamp and constant); a single
 *                       slice with taps_z = delta equals the 2-D separable
 *                       oracle; constant volumes; shifted deltas.
 *   conv2d_u8         : exact integer sums against numpy int64 slicing of the
 *                       padded image; delta taps reproduce the input; rounding
 *                       ties and saturation worked by hand; agreement with the
 *                       float oracle followed by the rounding rule.
 *   harris            : constant image gives R = 0 exactly; the linear ramp
 *                       a*x + b*y gives R = -k (64 (a^2+b^2))^2 away from the
 *                       edges; transposition; brute force on tiny images.
 *   nms               : constant gives an empty mask, a spike marks exactly one
 *                       pixel, a plateau keeps all members, brute force.
 *   bank adjoints     : the dot-product (adjoint) identity <Ax, g> = <x, A^T g>,
 *                       central finite differences (exact for this quadratic
 *                       loss up to rounding), delta filters, interior filter
 *                       gradient equal to a plain correlation.
 *   f16 / bf16 codecs : numpy's float16 and torch's bfloat16 conversions.
 * The paper itself prints no numeric outputs, so no pin is a paper value.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* closest in-range index along one axis (clamped boundary, Section 5) */
static inline long clampi(long i, long n) { return i < 0 ? 0 : (i > n - 1 ? n - 1 : i); }

/* clamped read of a W x H image stored row-major */
static inline double at(const double* X, long W, long H, long x, long y) {
    return X[clampi(y, H) * W + clampi(x, W)];
}

/* The two boundary conditions of Section 5 (Fig. 3): ORC_CLAMP reads the closest pixel
 * inside the image, ORC_CONSTANT returns the constant c for every read outside it. */
enum { ORC_CLAMP = 0, ORC_CONSTANT = 1 };

static inline int outside(long W, long H, long x, long y) { return x < 0 || x >= W || y < 0 || y >= H; }

static inline double at_b(const double* X, long W, long H, long x, long y, int border, double c) {
    if (border == ORC_CONSTANT && outside(W, H, x, y)) return c;
    return at(X, W, H, x, y);
}

/* ---------------------------------------------------------------- 2-D correlation
 * Y(x,y) = sum_{j=-r..r} sum_{i=-r..r} w[(j+r)(2r+1) + (i+r)] * X(x+i, y+j)
 * (non-separable convolution benchmark, Section 6; taps known at run time),
 * every read through the boundary condition. */
static double conv2d_px(const double* X, long W, long H, const double* w, int r, int border, double c,
                        long x, long y) {
    const int n = 2 * r + 1;
    double acc = 0.0;
    for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i)
            acc += w[(j + r) * n + (i + r)] * at_b(X, W, H, x + i, y + j, border, c);
    return acc;
}

EXPORT void orc_conv2d(const double* X, long W, long H, const double* w, int r, int border, double c,
                       double* Y, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            Y[y * W + x] = conv2d_px(X, W, H, w, r, border, c, x, y);
}

EXPORT void orc_conv2d_pts(const double* X, long W, long H, const double* w, int r, int border, double c,
                           const long* xs, const long* ys, long npts, double* out, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) out[p] = conv2d_px(X, W, H, w, r, border, c, xs[p], ys[p]);
}

/* ---------------------------------------------------------------- separable convolution
 * Row (R) kernel then column (C) kernel, as the paper's separable benchmark
 * splits it (Section 6, Table 2):
 *   T(x,y) = sum_i h[i+r] X(x+i, y)        Y(x,y) = sum_j v[j+r] T(x, y+j)
 * The intermediate T is kept in double.  The pair is the 2-D filter v (x) h on the
 * image extended by the boundary condition, so T is defined for every row the column
 * pass reads: under the clamped condition row y + j outside the image is row
 * clamp(y + j) (the closest pixel of the extended image); under the constant
 * condition every pixel of such a row is c, so T there is sum_i h[i+r] c. */
static double row_pass_px(const double* X, long W, long H, const double* h, int r, int border, double c,
                          long x, long y) {
    double acc = 0.0;
    for (int i = -r; i <= r; ++i) acc += h[i + r] * at_b(X, W, H, x + i, y, border, c);
    return acc;
}

static double row_pass_outside(const double* h, int r, double c) {
    double acc = 0.0;
    for (int i = -r; i <= r; ++i) acc += h[i + r] * c;
    return acc;
}

EXPORT void orc_conv_sep(const double* X, long W, long H, const double* h, const double* v, int r,
                         int border, double c, double* T, double* Y, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) T[y * W + x] = row_pass_px(X, W, H, h, r, border, c, x, y);
    const double t_out = row_pass_outside(h, r, c);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = -r; j <= r; ++j) {
                const long yy = y + j;
                const double t = (border == ORC_CONSTANT && (yy < 0 || yy >= H)) ? t_out : at(T, W, H, x, yy);
                acc += v[j + r] * t;
            }
            Y[y * W + x] = acc;
        }
}

/* the same two passes evaluated at single output pixels (row pass recomputed per column tap) */
EXPORT void orc_conv_sep_pts(const double* X, long W, long H, const double* h, const double* v, int r,
                             int border, double c, const long* xs, const long* ys, long npts, double* out,
                             int nthreads) {
    const double t_out = row_pass_outside(h, r, c);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) {
        const long x = xs[p], y = ys[p];
        double acc = 0.0;
        for (int j = -r; j <= r; ++j) {
            const long yy = y + j;
            const double t = (border == ORC_CONSTANT && (yy < 0 || yy >= H))
                                 ? t_out
                                 : row_pass_px(X, W, H, h, r, border, c, x, clampi(yy, H));
            acc += v[j + r] * t;
        }
        out[p] = acc;
    }
}

/* ---------------------------------------------------------------- 3-D separable correlation
 * The Image type also has 3-D indexing (Section 5).  A volume is stored slice after slice,
 * each slice row-major (x fastest).  The separable 3-D filter is the 3-D correlation with
 * taps hz (x) hy (x) hx on the volume extended by the boundary condition (per-axis clamp,
 * or the constant c outside):
 *   Y(x,y,z) = sum_{k,j,i} hz[k+r] hy[j+r] hx[i+r] X(x+i, y+j, z+k)
 * written out directly (no passes); the product of the three taps is formed first. */
static inline double at3(const double* X, long W, long H, long D, long x, long y, long z, int border, double c) {
    if (border == ORC_CONSTANT && (x < 0 || x >= W || y < 0 || y >= H || z < 0 || z >= D)) return c;
    return X[(clampi(z, D) * H + clampi(y, H)) * W + clampi(x, W)];
}

static double conv3d_sep_px(const double* X, long W, long H, long D, const double* hx, const double* hy,
                            const double* hz, int r, int border, double c, long x, long y, long z) {
    double acc = 0.0;
    for (int k = -r; k <= r; ++k)
        for (int j = -r; j <= r; ++j)
            for (int i = -r; i <= r; ++i)
                acc += (hz[k + r] * hy[j + r] * hx[i + r]) * at3(X, W, H, D, x + i, y + j, z + k, border, c);
    return acc;
}

EXPORT void orc_conv3d_sep(const double* X, long W, long H, long D, const double* hx, const double* hy,
                           const double* hz, int r, int border, double c, double* Y, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long z = 0; z < D; ++z)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x)
                Y[(z * H + y) * W + x] = conv3d_sep_px(X, W, H, D, hx, hy, hz, r, border, c, x, y, z);
}

EXPORT void orc_conv3d_sep_pts(const double* X, long W, long H, long D, const double* hx, const double* hy,
                               const double* hz, int r, int border, double c, const long* xs, const long* ys,
                               const long* zs, long npts, double* out, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p)
        out[p] = conv3d_sep_px(X, W, H, D, hx, hy, hz, r, border, c, xs[p], ys[p], zs[p]);
}

/* ---------------------------------------------------------------- 8-bit 2-D correlation
 * The non-separable benchmark of Section 6 runs on unsigned char pixels.  Taps are
 * signed 16-bit integers and the sum is exact integer arithmetic (here in 64 bits):
 *   S(x,y) = sum_{j,i} w[(j+r)(2r+1) + (i+r)] * X(x+i, y+j)
 *   Y(x,y) = min(max(floor((S + b) / 2^shift), 0), 255),  b = 2^(shift-1) (0 if shift = 0)
 * i.e. the fixed-point sum rounded to nearest with ties upward, then saturated to
 * 0..255.  Reads go through the boundary condition (constant c in 0..255). */
static inline long long floor_div_pow2(long long a, int shift) {
    const long long d = 1LL << shift;
    long long q = a / d;                       /* C division truncates toward zero */
    if (a % d != 0 && a < 0) q -= 1;
    return q;
}

static unsigned char conv2d_u8_px(const unsigned char* X, long W, long H, const int16_t* w, int r, int shift,
                                  int border, int c, long x, long y) {
    const int n = 2 * r + 1;
    long long acc = 0;
    for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i) {
            const long xx = x + i, yy = y + j;
            const long long p = (border == ORC_CONSTANT && outside(W, H, xx, yy))
                                    ? (long long)c
                                    : (long long)X[clampi(yy, H) * W + clampi(xx, W)];
            acc += (long long)w[(j + r) * n + (i + r)] * p;
        }
    const long long b = shift > 0 ? (1LL << (shift - 1)) : 0;
    const long long q = floor_div_pow2(acc + b, shift);
    return (unsigned char)(q < 0 ? 0 : (q > 255 ? 255 : q));
}

EXPORT void orc_conv2d_u8(const unsigned char* X, long W, long H, const int16_t* w, int r, int shift,
                          int border, int c, unsigned char* Y, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) Y[y * W + x] = conv2d_u8_px(X, W, H, w, r, shift, border, c, x, y);
}

EXPORT void orc_conv2d_u8_pts(const unsigned char* X, long W, long H, const int16_t* w, int r, int shift,
                              int border, int c, const long* xs, const long* ys, long npts, unsigned char* out,
                              int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) out[p] = conv2d_u8_px(X, W, H, w, r, shift, border, c, xs[p], ys[p]);
}

/* ---------------------------------------------------------------- Harris corner response
 * Harris corner detection is benchmarked in Section 6 as two kernels (Tables 4
 * and 5): a Sobel kernel producing the gradient images dx, dy, and a Harris
 * kernel reading dx, dy as Images (so its window reads are clamped on the
 * gradient images) and producing the response.
 *   Ix = sum s[j] d[i] X(x+i, y+j),  Iy = sum d[j] s[i] X(x+i, y+j),
 *        s = (1, 2, 1), d = (-1, 0, 1)
 *   A = Ix^2, B = Iy^2, C = Ix Iy
 *   Sxx = sum g[j] g[i] A(x+i, y+j)  (same for Syy from B, Sxy from C)
 *   R = Sxx Syy - Sxy^2 - k (Sxx + Syy)^2
 */
static const double SOB_S[3] = {1.0, 2.0, 1.0};
static const double SOB_D[3] = {-1.0, 0.0, 1.0};

static void sobel_px(const double* X, long W, long H, long x, long y, double* ix, double* iy) {
    double gx = 0.0, gy = 0.0;
    for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
            const double p = at(X, W, H, x + i, y + j);
            gx += SOB_S[j + 1] * SOB_D[i + 1] * p;
            gy += SOB_D[j + 1] * SOB_S[i + 1] * p;
        }
    *ix = gx;
    *iy = gy;
}

static void window_px(const double* A, const double* B, const double* C, long W, long H,
                      const double* g, int rg, long x, long y, double* sxx, double* syy, double* sxy) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int j = -rg; j <= rg; ++j)
        for (int i = -rg; i <= rg; ++i) {
            const double wgt = g[j + rg] * g[i + rg];
            a += wgt * at(A, W, H, x + i, y + j);
            b += wgt * at(B, W, H, x + i, y + j);
            c += wgt * at(C, W, H, x + i, y + j);
        }
    *sxx = a;
    *syy = b;
    *sxy = c;
}

static inline double response(double sxx, double syy, double sxy, double k) {
    const double tr = sxx + syy;
    return sxx * syy - sxy * sxy - k * tr * tr;
}

/* Full image.  work must hold 5*W*H doubles (Ix, Iy, A, B, C).  Sxx/Syy/Sxy may be NULL. */
EXPORT void orc_harris(const double* X, long W, long H, const double* g, int rg, double k, double* R,
                       double* Sxx, double* Syy, double* Sxy, double* work, int nthreads) {
    const long n = W * H;
    double *Ix = work, *Iy = work + n, *A = work + 2 * n, *B = work + 3 * n, *C = work + 4 * n;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double gx, gy;
            sobel_px(X, W, H, x, y, &gx, &gy);
            Ix[y * W + x] = gx;
            Iy[y * W + x] = gy;
        }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long q = 0; q < n; ++q) {
        A[q] = Ix[q] * Ix[q];
        B[q] = Iy[q] * Iy[q];
        C[q] = Ix[q] * Iy[q];
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double a, b, c;
            window_px(A, B, C, W, H, g, rg, x, y, &a, &b, &c);
            R[y * W + x] = response(a, b, c, k);
            if (Sxx) Sxx[y * W + x] = a;
            if (Syy) Syy[y * W + x] = b;
            if (Sxy) Sxy[y * W + x] = c;
        }
}

/* Magnitude scale of the response for normwise error measures: the same computation
 * with every term replaced by its absolute value (|Sobel taps| on |X|, non-negative
 * products, |window taps|), i.e.  Txx Tyy + Txy^2 + k (Txx + Tyy)^2  with
 * Txx = sum |g| |g| Gx^2, Gx = sum |s d| |X|.  A float32 evaluation of R differs from
 * the exact R by a small multiple of the unit roundoff times this scale, including
 * the cancellation inside the Sobel sums.  Not part of the method; test tolerance only. */
static void sobel_abs_px(const double* X, long W, long H, long x, long y, double* ax, double* ay) {
    double gx = 0.0, gy = 0.0;
    for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
            const double p = fabs(at(X, W, H, x + i, y + j));
            gx += fabs(SOB_S[j + 1] * SOB_D[i + 1]) * p;
            gy += fabs(SOB_D[j + 1] * SOB_S[i + 1]) * p;
        }
    *ax = gx;
    *ay = gy;
}

EXPORT void orc_harris_scale_pts(const double* X, long W, long H, const double* g, int rg, double k,
                                 const long* xs, const long* ys, long npts, double* S, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int j = -rg; j <= rg; ++j)
            for (int i = -rg; i <= rg; ++i) {
                double ax, ay;
                sobel_abs_px(X, W, H, clampi(xs[p] + i, W), clampi(ys[p] + j, H), &ax, &ay);
                const double wgt = fabs(g[j + rg] * g[i + rg]);
                a += wgt * ax * ax;
                b += wgt * ay * ay;
                c += wgt * ax * ay;
            }
        S[p] = a * b + c * c + fabs(k) * (a + b) * (a + b);
    }
}

/* Rounding-error bound of a float32 evaluation of the Harris chain (Section 6, Tables 4
 * and 5), at single pixels.  Not part of the method: the tests use it as the tolerance of
 * float32 responses and to find the pixels where rounding may decide a corner mask.
 *
 * Model: the input X holds float32 values (exact in double); every float32 operation
 * rounds to nearest with unit roundoff u = 2^-24 (an FMA rounds once); no underflow.
 * gamma(n) = n u / (1 - n u) bounds the relative error of a path of n roundings (Higham,
 * "Accuracy and Stability of Numerical Algorithms", Lemma 3.1), and a sum of products
 * evaluated in any order errs by at most gamma(depth) times the sum of |terms|.  The
 * bound holds for every evaluation order, so it serves each kernel variant.  Stages:
 *   Sobel    : 9 terms with exact coefficients (0, +-1, +-2), any order:
 *              |dIx| <= e_x = gamma(8) * sum |s d| |X|        (likewise Iy)
 *   products : A = Ix^2, B = Iy^2, C = Ix Iy, one rounding each:
 *              |dA| <= (2|Ix| + e_x) e_x + u (|Ix| + e_x)^2
 *              |dC| <= |Ix| e_y + |Iy| e_x + e_x e_y + u (|Ix| + e_x)(|Iy| + e_y)
 *   window   : S = sum g_j g_i A over (2r+1)^2 clamped positions; a path holds at most
 *              (2r+1)^2 + 1 roundings (tap product, term product, sum; a separable
 *              evaluation has 2 (2r+1) <= that), so with m = (2r+1)^2 + 1
 *              |dS| <= sum |g_j g_i| (|dA| + gamma(m) (|A| + |dA|))
 *   response : R(S + e) - R(S) expanded exactly,
 *              |dR| <= |Syy - 2k tr| d_xx + |Sxx - 2k tr| d_yy + 2 |Sxy| d_xy
 *                      + d_xx d_yy + d_xy^2 + |k| (d_xx + d_yy)^2
 *              plus its own evaluation (at most 5 roundings on a path, gamma(6) taken)
 *              on the magnitudes |S| + d:  gamma(6) (|Sxx||Syy| + Sxy^2 + |k| (|Sxx| + |Syy|)^2).
 * All quantities on the right are exact values computed here in double. */
static inline double gam(int n) {
    const double u = 0x1p-24;
    return n * u / (1.0 - n * u);
}

EXPORT void orc_harris_f32_bound_pts(const double* X, long W, long H, const double* g, int rg, double k,
                                     const long* xs, const long* ys, long npts, double* out, int nthreads) {
    const double u = 0x1p-24;
    const double gs = gam(8), gw = gam((2 * rg + 1) * (2 * rg + 1) + 1), gr = gam(6);
    const double ak = fabs(k);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) {
        double sxx = 0.0, syy = 0.0, sxy = 0.0, dxx = 0.0, dyy = 0.0, dxy = 0.0;
        for (int j = -rg; j <= rg; ++j)
            for (int i = -rg; i <= rg; ++i) {
                const long gxp = clampi(xs[p] + i, W), gyp = clampi(ys[p] + j, H);
                double ix, iy, ax, ay;
                sobel_px(X, W, H, gxp, gyp, &ix, &iy);
                sobel_abs_px(X, W, H, gxp, gyp, &ax, &ay);
                const double ex = gs * ax, ey = gs * ay;
                const double mx = fabs(ix) + ex, my = fabs(iy) + ey;
                const double ea = (2.0 * fabs(ix) + ex) * ex + u * mx * mx;
                const double eb = (2.0 * fabs(iy) + ey) * ey + u * my * my;
                const double ec = fabs(ix) * ey + fabs(iy) * ex + ex * ey + u * mx * my;
                const double wgt = g[j + rg] * g[i + rg], aw = fabs(wgt);
                sxx += wgt * ix * ix;
                syy += wgt * iy * iy;
                sxy += wgt * ix * iy;
                dxx += aw * (ea + gw * (ix * ix + ea));
                dyy += aw * (eb + gw * (iy * iy + eb));
                dxy += aw * (ec + gw * (fabs(ix * iy) + ec));
            }
        const double tr = sxx + syy;
        const double first = fabs(syy - 2.0 * k * tr) * dxx + fabs(sxx - 2.0 * k * tr) * dyy + 2.0 * fabs(sxy) * dxy;
        const double second = dxx * dyy + dxy * dxy + ak * (dxx + dyy) * (dxx + dyy);
        const double mxx = fabs(sxx) + dxx, myy = fabs(syy) + dyy, mxy = fabs(sxy) + dxy;
        const double rnd = gr * (mxx * myy + mxy * mxy + ak * (mxx + myy) * (mxx + myy));
        out[p] = first + second + rnd;
    }
}

/* Response at single pixels: gradients recomputed at every clamped window position. */
EXPORT void orc_harris_pts(const double* X, long W, long H, const double* g, int rg, double k,
                           const long* xs, const long* ys, long npts, double* R, double* Sxx,
                           double* Syy, double* Sxy, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int j = -rg; j <= rg; ++j)
            for (int i = -rg; i <= rg; ++i) {
                const long gxp = clampi(xs[p] + i, W), gyp = clampi(ys[p] + j, H);
                double ix, iy;
                sobel_px(X, W, H, gxp, gyp, &ix, &iy);
                const double wgt = g[j + rg] * g[i + rg];
                a += wgt * ix * ix;
                b += wgt * iy * iy;
                c += wgt * ix * iy;
            }
        R[p] = response(a, b, c, k);
        if (Sxx) Sxx[p] = a;
        if (Syy) Syy[p] = b;
        if (Sxy) Sxy[p] = c;
    }
}

/* ---------------------------------------------------------------- non-maximum suppression
 * M(x,y) = 1 iff R(x,y) > tau and R(x,y) >= R(x+i, y+j) for every (i,j) in the
 * (2r+1)^2 neighbourhood, reads clamped; otherwise 0.  R is taken as given (the
 * caller passes the exact values the kernel under test reads). */
static unsigned char nms_px(const double* R, long W, long H, int r, double tau, long x, long y) {
    const double c = R[y * W + x];
    if (!(c > tau)) return 0;
    for (int j = -r; j <= r; ++j)
        for (int i = -r; i <= r; ++i)
            if (!(c >= at(R, W, H, x + i, y + j))) return 0;
    return 1;
}

EXPORT void orc_nms(const double* R, long W, long H, int r, double tau, unsigned char* M, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) M[y * W + x] = nms_px(R, W, H, r, tau, x, y);
}

/* ---------------------------------------------------------------- differentiable filter bank
 * x: [N, H, W] (one channel), w: [F, 2r+1, 2r+1], y: [N, F, H, W], all row-major.
 *   y[n,f,y,x] = sum_{j,i} w[f,j,i] x[n, y+j, x+i]          (clamped correlation)
 *   L = sum (y - t)^2                                         dL/dy = 2 (y - t)
 *   dL/dx[n,q] = sum over (f, p, k) with clamp(p + k) = q of w[f,k] gy[n,f,p]
 *   dL/dw[f,k] = sum_{n,p} gy[n,f,p] x[n, clamp(p + k)]
 */
EXPORT void orc_bank_fwd(const double* x, const double* w, long N, long F, long H, long W, int r,
                         double* y, int nthreads) {
    const long hw = H * W, nk = (2 * r + 1) * (2 * r + 1);
    for (long n = 0; n < N; ++n)
        for (long f = 0; f < F; ++f)
            orc_conv2d(x + n * hw, W, H, w + f * nk, r, ORC_CLAMP, 0.0, y + (n * F + f) * hw, nthreads);
}

EXPORT double orc_sse_loss(const double* y, const double* t, long count, double* gy) {
    double L = 0.0;
    for (long q = 0; q < count; ++q) {
        const double d = y[q] - t[q];
        L += d * d;
        if (gy) gy[q] = 2.0 * d;
    }
    return L;
}

/* Input gradient by scatter: every forward read x[clamp(p+k)] sends w[f,k] gy[p] back to
 * the pixel it read.  Images are independent, so they are split across threads. */
EXPORT void orc_bank_bwd_input(const double* gy, const double* w, long N, long F, long H, long W, int r,
                               double* gx, int nthreads) {
    const long hw = H * W;
    const int n1 = 2 * r + 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long n = 0; n < N; ++n) {
        double* g = gx + n * hw;
        for (long q = 0; q < hw; ++q) g[q] = 0.0;
        for (long f = 0; f < F; ++f) {
            const double* gyf = gy + (n * F + f) * hw;
            const double* wf = w + f * n1 * n1;
            for (long y = 0; y < H; ++y)
                for (long x = 0; x < W; ++x)
                    for (int j = -r; j <= r; ++j)
                        for (int i = -r; i <= r; ++i)
                            g[clampi(y + j, H) * W + clampi(x + i, W)] += wf[(j + r) * n1 + (i + r)] * gyf[y * W + x];
        }
    }
}

/* Input gradient at single pixels q = (n, qx, qy), by the same definition: every (f, p, k)
 * whose clamped read lands on q.  Such p lie within 2r of q on each axis. */
EXPORT void orc_bank_bwd_input_pts(const double* gy, const double* w, long N, long F, long H, long W, int r,
                                   const long* ns, const long* xs, const long* ys, long npts, double* out,
                                   int nthreads) {
    const long hw = H * W;
    const int n1 = 2 * r + 1;
    (void)N;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long p = 0; p < npts; ++p) {
        const long n = ns[p], qx = xs[p], qy = ys[p];
        double acc = 0.0;
        for (long f = 0; f < F; ++f)
            for (long y = qy - 2 * r; y <= qy + 2 * r; ++y) {
                if (y < 0 || y >= H) continue;
                for (long x = qx - 2 * r; x <= qx + 2 * r; ++x) {
                    if (x < 0 || x >= W) continue;
                    for (int j = -r; j <= r; ++j) {
                        if (clampi(y + j, H) != qy) continue;
                        for (int i = -r; i <= r; ++i)
                            if (clampi(x + i, W) == qx)
                                acc += w[f * n1 * n1 + (j + r) * n1 + (i + r)] * gy[(n * F + f) * hw + y * W + x];
                    }
                }
            }
        out[p] = acc;
    }
}

/* Filter gradient; taps are independent sums, so they are split across threads.
 * (fk_lo, fk_hi) selects a range of the F*(2r+1)^2 flattened taps; pass 0, F*(2r+1)^2 for all. */
EXPORT void orc_bank_bwd_filter(const double* gy, const double* x, long N, long F, long H, long W, int r,
                                long fk_lo, long fk_hi, double* gw, int nthreads) {
    const long hw = H * W;
    const int n1 = 2 * r + 1;
    const long nk = (long)n1 * n1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic)
    for (long fk = fk_lo; fk < fk_hi; ++fk) {
        const long f = fk / nk, k = fk % nk;
        const int j = (int)(k / n1) - r, i = (int)(k % n1) - r;
        double acc = 0.0;
        for (long n = 0; n < N; ++n)
            for (long y = 0; y < H; ++y)
                for (long xx = 0; xx < W; ++xx)
                    acc += gy[(n * F + f) * hw + y * W + xx] * at(x + n * hw, W, H, xx + i, y + j);
        gw[fk - fk_lo] = acc;
    }
}

/* ---------------------------------------------------------------- storage formats
 * Decoders and round-to-nearest-even encoders for IEEE binary16 and bfloat16,
 * written from the format definitions (sign, biased exponent, fraction). */
EXPORT void orc_decode_f16(const uint16_t* in, double* out, long n) {
    for (long q = 0; q < n; ++q) {
        const unsigned b = in[q], s = b >> 15, e = (b >> 10) & 31u, m = b & 1023u;
        double v;
        if (e == 0) v = ldexp((double)m, -24);
        else if (e == 31) v = m ? NAN : INFINITY;
        else v = ldexp((double)(1024u + m), (int)e - 25);
        out[q] = s ? -v : v;
    }
}

EXPORT void orc_decode_bf16(const uint16_t* in, double* out, long n) {
    for (long q = 0; q < n; ++q) {
        const unsigned b = in[q], s = b >> 15, e = (b >> 7) & 255u, m = b & 127u;
        double v;
        if (e == 0) v = ldexp((double)m, -133);
        else if (e == 255) v = m ? NAN : INFINITY;
        else v = ldexp((double)(128u + m), (int)e - 134);
        out[q] = s ? -v : v;
    }
}

/* Round |v| to a binary format with `mb` fraction bits, exponent bias `bias` and `eb`
 * exponent bits, nearest-even, and return the bit pattern. */
static uint16_t encode_rne(double v, int mb, int eb, int bias) {
    const unsigned sign = signbit(v) ? 1u : 0u;
    const unsigned emax_field = (1u << eb) - 1u;
    double a = fabs(v);
    uint16_t bits;
    if (isnan(v)) {
        bits = (uint16_t)((emax_field << mb) | (1u << (mb - 1)));
        return (uint16_t)(bits | (sign << (mb + eb)));
    }
    const int emin = 1 - bias;                       /* smallest normal exponent */
    int e;
    if (a == 0.0) return (uint16_t)(sign << (mb + eb));
    frexp(a, &e);
    e -= 1;                                          /* a in [2^e, 2^(e+1)) */
    if (e < emin) e = emin;                          /* subnormal range shares the quantum of emin */
    const double quantum = ldexp(1.0, e - mb);
    const double q = a / quantum;                    /* exact: power-of-two scaling */
    double rq = floor(q);
    const double frac = q - rq;
    if (frac > 0.5 || (frac == 0.5 && fmod(rq, 2.0) != 0.0)) rq += 1.0;
    const double rv = rq * quantum;                  /* rounded magnitude, exact */
    /* re-encode rv */
    if (rv == 0.0) return (uint16_t)(sign << (mb + eb));
    int re;
    frexp(rv, &re);
    re -= 1;
    if (re > (int)emax_field - 1 - bias) {           /* overflow to infinity */
        bits = (uint16_t)(emax_field << mb);
    } else if (re < emin) {                          /* subnormal */
        bits = (uint16_t)(rv / ldexp(1.0, emin - mb));
    } else {
        const unsigned frac_bits = (unsigned)((rv / ldexp(1.0, re) - 1.0) * (double)(1u << mb));
        bits = (uint16_t)(((unsigned)(re + bias) << mb) | frac_bits);
    }
    return (uint16_t)(bits | (sign << (mb + eb)));
}

EXPORT void orc_encode_f16(const double* in, uint16_t* out, long n) {
    for (long q = 0; q < n; ++q) out[q] = encode_rne(in[q], 10, 5, 15);
}

EXPORT void orc_encode_bf16(const double* in, uint16_t* out, long n) {
    for (long q = 0; q < n; ++q) out[q] = encode_rne(in[q], 7, 8, 127);
}
