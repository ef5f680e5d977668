// Differentiable filter bank: F filters of radius r over N single-channel images
// (clamped correlation) and its adjoints.  Dense NCHW float32 tensors.
//
//   forward      y[n,f,p]  = sum_k w[f,k] x[n, clamp(p+k)]
//   input grad   gx[n,q]   = sum_{f,p,k : clamp(p+k) = q} w[f,k] gy[n,f,p]
//                          = sum_{u : clamp(u) = q} z[n,u],
//                z[n,u]    = sum_f sum_k w[f,k] gy0[n,f,u-k]       (gy0: gy extended by zero)
//                i.e. a correlation of the zero-padded gy with the flipped filters on
//                the padded grid, folded back onto the edge pixels it was clamped to.
//   filter grad  gw[f,k]   = sum_{n,p} gy[n,f,p] x[n, clamp(p+k)]
//
// Kernels
//   bank_fwd       : 64x64 output tile per 256-lane work-group; the x tile with its
//                    r halo is staged in LDS once and reused by all F filters; each
//                    lane keeps a 4x4 accumulator block (input-row-outer order).
//   bank_bwd_in    : same tiling; for each filter the gy tile (zero outside the image)
//                    is staged and correlated with the flipped filter; the F sums
//                    accumulate in registers and are stored once.
//   bank_bwd_edge  : recomputes the border pixels, where the clamp folds padded positions
//                    onto q, as a correlation of gy with box sums of the taps; one
//                    work-group per 256-pixel border segment, gy strip staged in LDS.
//   bank_bwd_w1/w2 : filter gradient.  Stage 1: one wave per (image, 32x64 tile,
//                    filter) accumulates all (2r+1)^2 taps over its 2048 pixels
//                    (column-walk register reuse), reduces across the wave with a
//                    butterfly, and writes one partial per tap.  Stage 2 sums the
//                    partials of each (f, tap) in a fixed order: deterministic.
//   bank_bwd_w4    : stage 1 with four filters per work-group sharing one staged x
//                    tile (one wave each), over 64 x 64 or 64 x 256 pixels (four
//                    staged 64-row sub-tiles before the single cross-lane reduction).
#include "corr_tile.hpp"
#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "tile_stage.hpp"

namespace icl {
namespace {

constexpr int BT = 64;           // fwd / bwd_in tile side
constexpr int BPX = 4, BPY = 4;  // per-lane accumulator block (16 x 16 lanes)

template <int R> struct BankTile {
    static constexpr int RA = (R + 3) & ~3;
    static constexpr int LW = BT + 2 * RA;
    static constexpr int NR = BT + 2 * R;
    static constexpr int WIN = BPX + 2 * RA;
};

// Stage NR rows x LWS columns of a dense W-wide plane, top-left pixel (xs, ys), clamped, into
// s[NR * LW] (row stride LW >= LWS).  A tile inside the image in x with 16-byte aligned rows
// issues all its float4 loads before the LDS writes (a load-then-write loop would wait on each
// load in turn); edge tiles go element by element.
template <int NR, int LW, int LWS = LW>
__device__ __forceinline__ void stage_clamped(const float* __restrict__ xp, int W, int H, int xs, int ys,
                                              float* __restrict__ s) {
    const int tid = threadIdx.x;
    if ((W & 3) == 0 && ((uintptr_t)xp & 15) == 0 && (xs & 3) == 0 && xs >= 0 && xs + LWS <= W) {
        static_assert(LW % 4 == 0 && LWS % 4 == 0, "vector staging needs whole float4 rows");
        constexpr int C4 = LWS / 4, NCH = NR * C4, PER = (NCH + 255) / 256;
        v4f v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            v[i] = *reinterpret_cast<const v4f*>(xp + (size_t)clampi(ys + rr, H) * W + xs + 4 * c4);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            lds4(&s[rr * LW + 4 * c4], v[i]);
        }
        return;
    }
    for (int idx = tid; idx < NR * LWS; idx += 256) {   // edge tiles
        const int rr = idx / LWS, c = idx - rr * LWS;
        s[rr * LW + c] = xp[(size_t)clampi(ys + rr, H) * W + clampi(xs + c, W)];
    }
}

// Stage rows y0-R .. y0+BT+R-1 and columns x0-RA .. x0+BT+RA-1 of a dense W-wide
// plane into LDS.  ZERO_PAD: outside pixels read as 0; otherwise clamped.
template <int R, bool ZERO_PAD>
__device__ __forceinline__ void stage_plane(const float* __restrict__ plane, int W, int H, int x0, int y0,
                                            bool vec, float* __restrict__ s) {
    using G = BankTile<R>;
    constexpr int LW = G::LW, NR = G::NR, RA = G::RA;
    const int tid = threadIdx.x;
    if (vec && x0 - RA >= 0 && x0 + BT + RA <= W) {
        constexpr int C4 = LW / 4;
        for (int idx = tid; idx < NR * C4; idx += 256) {
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int yy = y0 - R + rr;
            v4f v;
            if (ZERO_PAD && (yy < 0 || yy >= H)) v = mk4(0.f, 0.f, 0.f, 0.f);
            else v = *reinterpret_cast<const v4f*>(plane + (size_t)clampi(yy, H) * W + (x0 - RA + 4 * c4));
            lds4(&s[rr * LW + 4 * c4], v);
        }
    } else {
        for (int idx = tid; idx < NR * LW; idx += 256) {
            const int rr = idx / LW, c = idx - rr * LW;
            const int yy = y0 - R + rr, xx = x0 - RA + c;
            float v;
            if (ZERO_PAD && (yy < 0 || yy >= H || xx < 0 || xx >= W)) v = 0.f;
            else v = plane[(size_t)clampi(yy, H) * W + clampi(xx, W)];
            s[rr * LW + c] = v;
        }
    }
}

// acc += correlation of the staged tile with taps wf (flat (2r+1)^2, row major);
// FLIP reads the taps reversed (the adjoint's flipped filter).
template <int R, bool FLIP>
__device__ __forceinline__ void corr_block(const float* __restrict__ s, const float* __restrict__ wf,
                                           float (&acc)[BPY][BPX]) {
    using G = BankTile<R>;
    constexpr int LW = G::LW, RA = G::RA, WIN = G::WIN, N = 2 * R + 1;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const float* base = s + (ty * BPY) * LW + tx * BPX;
#pragma unroll 1
    for (int q = 0; q < BPY + 2 * R; ++q) {
        float win[WIN];
#pragma unroll
        for (int m = 0; m < WIN / 4; ++m) {
            const v4f v = lds4(base + q * LW + 4 * m);
            win[4 * m] = v.x; win[4 * m + 1] = v.y; win[4 * m + 2] = v.z; win[4 * m + 3] = v.w;
        }
#pragma unroll
        for (int py = 0; py < BPY; ++py) {
            const int j = q - py;
            if (j < 0 || j >= N) continue;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const float c = FLIP ? wf[N * N - 1 - (j * N + i)] : wf[j * N + i];
#pragma unroll
                for (int px = 0; px < BPX; ++px) acc[py][px] = fmaf(c, win[RA - R + px + i], acc[py][px]);
            }
        }
    }
}

__device__ __forceinline__ void store_block(float* __restrict__ plane, int W, int H, int x0, int y0, bool vec,
                                            const float (&acc)[BPY][BPX]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int xb = x0 + tx * BPX;
#pragma unroll
    for (int py = 0; py < BPY; ++py) {
        const int y = y0 + ty * BPY + py;
        if (y >= H) break;
        float* row = plane + (size_t)y * W;
        if (vec && xb + BPX <= W) {
            *reinterpret_cast<v4f*>(row + xb) = mk4(acc[py][0], acc[py][1], acc[py][2], acc[py][3]);
        } else {
#pragma unroll
            for (int px = 0; px < BPX; ++px)
                if (xb + px < W) row[xb + px] = acc[py][px];
        }
    }
}

template <int R>
__global__ __launch_bounds__(256) void bank_fwd_k(const float* __restrict__ x, const float* __restrict__ w,
                                                  float* __restrict__ y, int F, int H, int W, int tiles_x,
                                                  int tiles_img, int vec) {
    using G = BankTile<R>;
    __shared__ __attribute__((aligned(16))) float s[G::NR * G::LW];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int n = (int)(t / (unsigned)tiles_img), ti = (int)(t % (unsigned)tiles_img);
    const int x0 = (ti % tiles_x) * BT, y0 = (ti / tiles_x) * BT;
    const size_t hw = (size_t)H * W;
    stage_plane<R, false>(x + (size_t)n * hw, W, H, x0, y0, vec, s);
    __syncthreads();
    constexpr int NK = (2 * R + 1) * (2 * R + 1);
#pragma unroll 1
    for (int f = 0; f < F; ++f) {
        float acc[BPY][BPX] = {};
        corr_block<R, false>(s, w + (size_t)f * NK, acc);
        store_block(y + ((size_t)n * F + f) * hw, W, H, x0, y0, vec, acc);
    }
}

// The adjoints' output factor: *scale when given (an upstream gradient on the loss), else 1.
// Multiplying by 1.0f is exact, so without a factor the outputs are unchanged bit for bit.
__device__ __forceinline__ float out_scale(const float* __restrict__ scale) { return scale ? *scale : 1.f; }

__device__ __forceinline__ void scale_acc(float (&acc)[BPY][BPX], float sc) {
#pragma unroll
    for (int py = 0; py < BPY; ++py)
#pragma unroll
        for (int px = 0; px < BPX; ++px) acc[py][px] *= sc;
}

template <int R>
__global__ __launch_bounds__(256) void bank_bwd_in_k(const float* __restrict__ gy, const float* __restrict__ w,
                                                     float* __restrict__ gx, int F, int H, int W, int tiles_x,
                                                     int tiles_img, int vec, const float* __restrict__ scale) {
    using G = BankTile<R>;
    __shared__ __attribute__((aligned(16))) float s[G::NR * G::LW];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int n = (int)(t / (unsigned)tiles_img), ti = (int)(t % (unsigned)tiles_img);
    const int x0 = (ti % tiles_x) * BT, y0 = (ti / tiles_x) * BT;
    const size_t hw = (size_t)H * W;
    constexpr int NK = (2 * R + 1) * (2 * R + 1);
    float acc[BPY][BPX] = {};
#pragma unroll 1
    for (int f = 0; f < F; ++f) {
        if (f) __syncthreads();
        stage_plane<R, true>(gy + ((size_t)n * F + f) * hw, W, H, x0, y0, vec, s);
        __syncthreads();
        corr_block<R, true>(s, w + (size_t)f * NK, acc);
    }
    scale_acc(acc, out_scale(scale));
    store_block(gx + (size_t)n * hw, W, H, x0, y0, vec, acc);
}

// Border pixels.  For a pixel q on the image border the clamp maps the whole interval
// S_x(q) x S_y(q) of padded positions onto q (S_x = [-r, 0] on the left edge, [W-1, W-1+r]
// on the right, {qx} elsewhere; the same for y), so
//   gx[n,q] = sum_f sum_p gy[n,f,p] * B_f(q,p),   B_f(q,p) = sum_{k in (S(q) - p), |k| <= r} w[f,k],
// a correlation of gy with box sums of the taps.  Each box sum is taken directly over its
// own taps (no differences of prefix sums), so its rounding is bounded by the box's own
// magnitude.  The value replaces what the interior kernel wrote at q.
//
// One work-group per (image, side, 256-pixel segment): top and bottom rows (corners
// included), then the left and right columns without their end rows.  For each filter the
// r+1 deep strip of gy along the segment (plus r on each end, zero outside the image) is
// staged in LDS, row-major along the edge so that the loads stay contiguous.
constexpr int EDGE_SEG = 256;

struct EdgeSegments {
    int top, bottom, left, right;
    int per_image() const { return top + bottom + left + right; }
};

EdgeSegments edge_segments(int W, int H) {
    EdgeSegments e;
    e.top = (W + EDGE_SEG - 1) / EDGE_SEG;
    e.bottom = H > 1 ? e.top : 0;                                   // H == 1: the top row is the bottom row
    e.left = H > 2 ? (H - 2 + EDGE_SEG - 1) / EDGE_SEG : 0;
    e.right = (H > 2 && W > 1) ? e.left : 0;                        // W == 1: the left column is the right one
    return e;
}

template <int R>
__global__ __launch_bounds__(256) void bank_bwd_edge_k(const float* __restrict__ gy, const float* __restrict__ w,
                                                       float* __restrict__ gx, int F, int H, int W, int top,
                                                       int bottom, int left, int per_img,
                                                       const float* __restrict__ scale) {
    constexpr int N = 2 * R + 1, L = EDGE_SEG + 2 * R;
    __shared__ float wl[64 * N * N];
    __shared__ float strip[L * (R + 1)];
    __shared__ float tab[(R + 1) * N];   // this side's one-axis box sums of the current filter
    __shared__ float ctab[2][(R + 1) * (R + 1)];   // 2-D box sums of the left / right corner
    for (int i = threadIdx.x; i < F * N * N; i += 256) wl[i] = w[i];
    const int n = blockIdx.x / per_img;
    int s = blockIdx.x - n * per_img, side, a0;
    if (s < top) { side = 0; a0 = s * EDGE_SEG; }
    else if ((s -= top) < bottom) { side = 1; a0 = s * EDGE_SEG; }
    else if ((s -= bottom) < left) { side = 2; a0 = 1 + s * EDGE_SEG; }
    else { s -= left; side = 3; a0 = 1 + s * EDGE_SEG; }
    const int along = side < 2 ? W : H;
    const int D = min(R + 1, side < 2 ? H : W);                      // strip depth
    const int a = a0 + (int)threadIdx.x;
    const bool active = a < (side < 2 ? W : H - 1);
    // (along, depth) -> pixel
    auto pixel = [&](int aa, int d, int& x, int& y) {
        switch (side) {
            case 0: x = aa; y = d; break;
            case 1: x = aa; y = H - 1 - d; break;
            case 2: x = d; y = aa; break;
            default: x = W - 1 - d; y = aa; break;
        }
    };
    int qx, qy;
    pixel(a, 0, qx, qy);
    const int sxl = qx == 0 ? -R : qx, sxh = qx == W - 1 ? W - 1 + R : qx;
    const int syl = qy == 0 ? -R : qy, syh = qy == H - 1 ? H - 1 + R : qy;
    const int pxl = max(sxl - R, 0), pxh = min(sxh + R, W - 1);
    const int pyl = max(syl - R, 0), pyh = min(syh + R, H - 1);
    // Fast path: a pixel that is on exactly one edge of an image at least two pixels across
    // that edge.  Its box is then a one-axis interval at depth d from the edge times a
    // single tap across it, so B_f(q, p) = tab[d][r - e] with e the offset of p along the
    // edge; tab is summed once per filter.  Corners use a table of 2-D boxes; only one-row
    // and one-column images take the general loop.
    const bool fast = side < 2 ? (H > 1 && qx != 0 && qx != W - 1) : W > 1;
    // corner pixels of an image at least two pixels in each direction: B_f(q, p) is a box
    // at depth (dy, dx) from both edges, ctab[c][dy][dx] (c = 0 left, 1 right corner)
    const bool corner = side < 2 && H > 1 && W > 1 && (qx == 0 || qx == W - 1);
    const bool has_left = side < 2 && H > 1 && W > 1 && a0 == 0;
    const bool has_right = side < 2 && H > 1 && W > 1 && W - 1 - a0 < EDGE_SEG;
    const int Dx = min(R + 1, W);
    const int t = (int)threadIdx.x;
    const size_t hw = (size_t)H * W;
    // The strip of filter f+1 is loaded into registers while filter f is computed (thread
    // t holds strip entries t, t + 256, ...), so the global loads of the whole walk overlap.
    constexpr int NPRE = (L * (R + 1) + 255) / 256;
    float pre[NPRE];
    auto fetch = [&](int f) {
        const float* g = gy + ((size_t)n * F + f) * hw;
#pragma unroll
        for (int u = 0; u < NPRE; ++u) {
            const int idx = t + 256 * u;
            const int ai = idx / D, d = idx - ai * D, aa = a0 - R + ai;
            float v = 0.f;
            if (idx < L * D && aa >= 0 && aa < along) {
                int x, y;
                pixel(aa, d, x, y);
                v = g[(size_t)y * W + x];
            }
            pre[u] = v;
        }
    };
    fetch(0);
    float acc = 0.f;
    for (int f = 0; f < F; ++f) {
        __syncthreads();   // taps staged; previous strip and table consumed
#pragma unroll
        for (int u = 0; u < NPRE; ++u)
            if (t + 256 * u < L * D) strip[t + 256 * u] = pre[u];
        if (f + 1 < F) fetch(f + 1);
        const float* wf = wl + f * N * N;
        if (t < (R + 1) * N) {
            // top: sum over rows ky = -r .. -d; bottom: ky = d .. r; left / right: the same
            // over columns.  Each box is summed directly, in ascending tap order.
            const int d = t / N, k = t - d * N;
            const int lo = side == 0 || side == 2 ? 0 : R + d, hi = side == 0 || side == 2 ? R - d : 2 * R;
            float b = 0.f;
            for (int m = lo; m <= hi; ++m) b += side < 2 ? wf[m * N + k] : wf[k * N + m];
            tab[t] = b;
        }
        {
            // corner boxes: rows -r .. -dy (top) or dy .. r (bottom), columns -r .. -dx
            // (left corner) or dx .. r (right corner), summed directly
            const int u = t - 64, c = u / ((R + 1) * (R + 1)), e = u - c * (R + 1) * (R + 1);
            if (u >= 0 && c < 2 && (c == 0 ? has_left : has_right)) {
                const int dy = e / (R + 1), dx = e - dy * (R + 1);
                const int rlo = side == 0 ? 0 : R + dy, rhi = side == 0 ? R - dy : 2 * R;
                const int clo = c == 0 ? 0 : R + dx, chi = c == 0 ? R - dx : 2 * R;
                float b = 0.f;
                for (int m = rlo; m <= rhi; ++m)
                    for (int l = clo; l <= chi; ++l) b += wf[m * N + l];
                ctab[c][e] = b;
            }
        }
        __syncthreads();
        if (!active) continue;
        if (fast) {
            for (int d = 0; d < D; ++d) {
#pragma unroll
                for (int e = -R; e <= R; ++e) acc = fmaf(strip[(t + e + R) * D + d], tab[d * N + R - e], acc);
            }
            continue;
        }
        if (corner) {
            const int c = qx == 0 ? 0 : 1;
            for (int dy = 0; dy < D; ++dy)
                for (int dx = 0; dx < Dx; ++dx) {
                    const int px = c == 0 ? dx : W - 1 - dx;
                    acc = fmaf(strip[(px - a0 + R) * D + dy], ctab[c][dy * (R + 1) + dx], acc);
                }
            continue;
        }
        for (int py = pyl; py <= pyh; ++py) {
            const int kyl = max(syl - py, -R), kyh = min(syh - py, R);
            for (int px = pxl; px <= pxh; ++px) {
                const int kxl = max(sxl - px, -R), kxh = min(sxh - px, R);
                float b = 0.f;
                for (int ky = kyl; ky <= kyh; ++ky)
                    for (int kx = kxl; kx <= kxh; ++kx) b += wf[(ky + R) * N + kx + R];
                int ai, d;
                switch (side) {
                    case 0: ai = px - a0 + R; d = py; break;
                    case 1: ai = px - a0 + R; d = H - 1 - py; break;
                    case 2: ai = py - a0 + R; d = px; break;
                    default: ai = py - a0 + R; d = W - 1 - px; break;
                }
                acc = fmaf(strip[ai * D + d], b, acc);
            }
        }
    }
    if (active) gx[(size_t)n * hw + (size_t)qy * W + qx] = acc * out_scale(scale);
}

template <int R>
hipError_t launch_edge(const BankArgs& a) {
    const EdgeSegments e = edge_segments(a.w, a.h);
    const int per = e.per_image();
    hipLaunchKernelGGL(bank_bwd_edge_k<R>, dim3((unsigned)(a.n * per)), dim3(256), 0, a.st, a.a, a.b, a.out, a.f,
                       a.h, a.w, e.top, e.bottom, e.left, per, a.scale);
    return hipGetLastError();
}

// ------------------------------------------------------------------ filter gradient
constexpr int GW_TW = 32, GW_TH = 64, GW_CH = 16;   // tile 32 cols x 64 rows, row chunks of 16

template <int R> struct GwTile {
    static constexpr int RA = (R + 3) & ~3;
    static constexpr int LW = GW_TW + 2 * RA;
    static constexpr int NR = GW_TH + 2 * R;
};

template <int R>
__global__ __launch_bounds__(64) void bank_bwd_w1_k(const float* __restrict__ gy, const float* __restrict__ x,
                                                    float* __restrict__ part, int F, int H, int W, int tiles_x,
                                                    int tiles_img, int ntiles) {
    using G = GwTile<R>;
    constexpr int N = 2 * R + 1, LW = G::LW, NR = G::NR, RA = G::RA;
    __shared__ __attribute__((aligned(16))) float s[NR * LW];
    // block -> (tile, filter); the F blocks of one tile are consecutive logical ids, kept on one XCD
    const unsigned id = xcd_remap(blockIdx.x, gridDim.x);
    const int f = (int)(id % (unsigned)F);
    const int tile = (int)(id / (unsigned)F);
    const int n = tile / tiles_img, ti = tile % tiles_img;
    const int x0 = (ti % tiles_x) * GW_TW, y0 = (ti / tiles_x) * GW_TH;
    const size_t hw = (size_t)H * W;
    const float* xp = x + (size_t)n * hw;
    const int lane = threadIdx.x;
    for (int idx = lane; idx < NR * LW; idx += 64) {
        const int rr = idx / LW, c = idx - rr * LW;
        s[idx] = xp[(size_t)clampi(y0 - R + rr, H) * W + clampi(x0 - RA + c, W)];
    }
    __syncthreads();
    const float* g = gy + ((size_t)n * F + f) * hw;
    const int col = lane & 31, half = lane >> 5;
    const int gx_ = x0 + col;
    float acc[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) acc[j][i] = 0.f;
#pragma unroll 1
    for (int c = 0; c < GW_TH / 2 / GW_CH; ++c) {
        const int r0 = half * (GW_TH / 2) + c * GW_CH;   // first tile row of this chunk
        float gv[GW_CH];
#pragma unroll
        for (int py = 0; py < GW_CH; ++py) {
            const int yy = y0 + r0 + py;
            gv[py] = (gx_ < W && yy < H) ? g[(size_t)yy * W + gx_] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float cv[GW_CH + 2 * R];
#pragma unroll
            for (int m = 0; m < GW_CH + 2 * R; ++m) cv[m] = s[(r0 + m) * LW + col + RA - R + i];
#pragma unroll
            for (int j = 0; j < N; ++j)
#pragma unroll
                for (int py = 0; py < GW_CH; ++py) acc[j][i] = fmaf(gv[py], cv[py + j], acc[j][i]);
        }
    }
    // butterfly over the wave (fixed order), lane 0 writes the (f, tile) partials
    float* out = part + (size_t)f * N * N * ntiles + tile;
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float v = acc[j][i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) out[(size_t)(j * N + i) * ntiles] = v;
        }
}

// gw[f,k] = sum over tiles of part[f][k][tile], fixed-order tree per (f, k)
__global__ __launch_bounds__(256) void bank_bwd_w2_k(const float* __restrict__ part, float* __restrict__ gw,
                                                     int ntiles, const float* __restrict__ scale) {
    __shared__ float red[256];
    const float* p = part + (size_t)blockIdx.x * ntiles;
    float v = 0.f;
    for (int t = threadIdx.x; t < ntiles; t += 256) v += p[t];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) gw[blockIdx.x] = red[0] * out_scale(scale);
}

// ------------------------------------------------------------------ plain baselines
// One output per lane, runtime loops, clamped reads straight from global memory.
__global__ __launch_bounds__(256) void bank_fwd_plain_k(const float* __restrict__ x, const float* __restrict__ w,
                                                        float* __restrict__ y, int N, int F, int H, int W, int r) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long hw = (long long)H * W;
    if (i >= (long long)N * F * hw) return;
    const int n = (int)(i / (F * hw));
    const int f = (int)((i / hw) % F);
    const int p = (int)(i % hw), py = p / W, px = p - py * W;
    const int nk = 2 * r + 1;
    const float* xp = x + (size_t)n * hw;
    const float* wf = w + (size_t)f * nk * nk;
    float acc = 0.f;
    for (int j = -r; j <= r; ++j)
        for (int q = -r; q <= r; ++q)
            acc = fmaf(wf[(j + r) * nk + (q + r)], xp[(size_t)clampi(py + j, H) * W + clampi(px + q, W)], acc);
    y[i] = acc;
}

// Input gradient straight from the adjoint's definition: gx[q] = sum over padded u with
// clamp(u) = q of z[u], z[u] = sum_f sum_k w[f,k] gy0[f, u-k].
__global__ __launch_bounds__(256) void bank_bwd_in_plain_k(const float* __restrict__ gy, const float* __restrict__ w,
                                                           float* __restrict__ gx, int N, int F, int H, int W, int r,
                                                           const float* __restrict__ scale) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long hw = (long long)H * W;
    if (i >= (long long)N * hw) return;
    const int n = (int)(i / hw);
    const int p = (int)(i % hw), qy = p / W, qx = p - qy * W;
    const int lox = (qx == 0) ? -r : qx, hix = (qx == W - 1) ? W - 1 + r : qx;
    const int loy = (qy == 0) ? -r : qy, hiy = (qy == H - 1) ? H - 1 + r : qy;
    const int nk = 2 * r + 1;
    float acc = 0.f;
    for (int uy = loy; uy <= hiy; ++uy)
        for (int ux = lox; ux <= hix; ++ux)
            for (int f = 0; f < F; ++f) {
                const float* g = gy + ((size_t)n * F + f) * hw;
                const float* wf = w + (size_t)f * nk * nk;
                for (int j = -r; j <= r; ++j) {
                    const int sy = uy - j;
                    if (sy < 0 || sy >= H) continue;
                    for (int q = -r; q <= r; ++q) {
                        const int sx = ux - q;
                        if (sx < 0 || sx >= W) continue;
                        acc = fmaf(wf[(j + r) * nk + (q + r)], g[(size_t)sy * W + sx], acc);
                    }
                }
            }
    gx[i] = acc * out_scale(scale);
}

// ------------------------------------------------------------------ persistent, prefetching, taps in LDS
constexpr int PERS_FMAX = 16;   // filters whose taps fit the static LDS table

// Target block of the fused loss: the lane's BPY x BPX pixels of plane `tg` (0 outside).
__device__ __forceinline__ void load_block(const float* __restrict__ plane, int W, int H, int x0, int y0, bool vec,
                                           float (&v)[BPY][BPX]) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int xb = x0 + tx * BPX;
#pragma unroll
    for (int py = 0; py < BPY; ++py) {
        const int y = y0 + ty * BPY + py;
        const float* row = plane + (size_t)(y < H ? y : 0) * W;
        if (y < H && vec && xb + BPX <= W) {
            const v4f q = *reinterpret_cast<const v4f*>(row + xb);
            v[py][0] = q.x; v[py][1] = q.y; v[py][2] = q.z; v[py][3] = q.w;
        } else {
#pragma unroll
            for (int px = 0; px < BPX; ++px) v[py][px] = (y < H && xb + px < W) ? row[xb + px] : 0.f;
        }
    }
}

// Loss epilogue of the fused forward: d = y - t on the lane's in-image pixels; adds the
// block's sum of d^2 (float32 over these <= 16 terms) to `sq`, writes gy = 2 d and y where
// the pointers are non-null.  2 d is the same float32 product as the stand-alone loss.
__device__ __forceinline__ void sse_block(float* __restrict__ gyp, float* __restrict__ yp, int W, int H, int x0,
                                          int y0, bool vec, const float (&acc)[BPY][BPX],
                                          const float (&tv)[BPY][BPX], double& sq) {
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int xb = x0 + tx * BPX;
    float s = 0.f;
#pragma unroll
    for (int py = 0; py < BPY; ++py) {
        const int y = y0 + ty * BPY + py;
        if (y >= H) break;
        const size_t off = (size_t)y * W + xb;
        float d[BPX];
#pragma unroll
        for (int px = 0; px < BPX; ++px) d[px] = acc[py][px] - tv[py][px];
        if (vec && xb + BPX <= W) {
#pragma unroll
            for (int px = 0; px < BPX; ++px) s = fmaf(d[px], d[px], s);
            if (gyp) *reinterpret_cast<v4f*>(gyp + off) = 2.f * mk4(d[0], d[1], d[2], d[3]);
            if (yp) *reinterpret_cast<v4f*>(yp + off) = mk4(acc[py][0], acc[py][1], acc[py][2], acc[py][3]);
        } else {
#pragma unroll
            for (int px = 0; px < BPX; ++px)
                if (xb + px < W) {
                    s = fmaf(d[px], d[px], s);
                    if (gyp) gyp[off + px] = 2.f * d[px];
                    if (yp) yp[off + px] = acc[py][px];
                }
        }
    }
    sq += (double)s;
}

// Work-group sum of one double per lane into part[blockIdx.x], through LDS scratch of
// at least 256 doubles (fixed tree order).
__device__ __forceinline__ void block_sum_store(double v, double* __restrict__ red, double* __restrict__ part) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// SSE: the forward fused with the sum-of-squares loss against tg (y and gy optional, the
// block's partial sum of (y - t)^2 to part[blockIdx.x]); otherwise the plain forward into y.
template <int R, bool SSE, bool TPRE>
__device__ __forceinline__ void bank_fwd_pers_body(const float* __restrict__ x, const float* __restrict__ w,
                                                   float* __restrict__ y, const float* __restrict__ tg,
                                                   float* __restrict__ gy, double* __restrict__ part, int F, int H,
                                                   int W, int tiles_x, int tiles_img, int ntiles, int vec) {
    using G = BankTile<R>;
    constexpr int LW = G::LW, NR = G::NR, RA = G::RA, N = 2 * R + 1, NP = (N + 3) & ~3;
    static_assert(2 * NR * LW * sizeof(float) >= 256 * sizeof(double), "the x tiles double as reduction scratch");
    // two x tiles: the next tile is staged into the idle one while all F filters run on the other
    __shared__ __attribute__((aligned(16))) float s[2][NR * LW];
    __shared__ __attribute__((aligned(16))) float wl[PERS_FMAX * N * NP];
    taps_to_lds<R, false>(w, F, wl);
    const size_t hw = (size_t)H * W;
    Stage<F32, NR, LW> st;
    auto fetch = [&](int t) {
        const int n = t / tiles_img, ti = t - n * tiles_img;
        int x0, y0;
        tile_origin(ti, tiles_x, BT, BT, x0, y0);
        st.load(x + (size_t)n * hw, (size_t)W * 4, W, H, x0 - RA, y0 - R, vec);
    };
    const BandWalk walk(tiles_x, ntiles / tiles_x);   // images stacked vertically
    int t = walk.tile(0);
    if (t >= 0) {
        fetch(t);
        st.store(s[0]);
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    int cur = 0;
    double sq = 0.0;
    for (int k = 0; t >= 0; ++k) {
        const int n = t / tiles_img, ti = t - n * tiles_img;
        int x0, y0;
        tile_origin(ti, tiles_x, BT, BT, x0, y0);
        const int tn = walk.tile(k + 1);
        if (tn >= 0) fetch(tn);
#pragma unroll 1
        for (int f = 0; f < F; ++f) {
            const size_t plane = ((size_t)n * F + f) * hw;
            float tv[BPY][BPX];
            if constexpr (SSE && TPRE) load_block(tg + plane, W, H, x0, y0, vec, tv);   // in flight during the FMAs
            float acc[BPY][BPX] = {};
            corr_rows<R, BPX, BPY, LW>(&s[cur][(ty * BPY) * LW + tx * BPX], &wl[f * N * NP], acc);
            if constexpr (SSE && !TPRE) {
                __builtin_amdgcn_sched_barrier(0);   // keep the target loads (and their registers) after the FMAs
                load_block(tg + plane, W, H, x0, y0, vec, tv);
            }
            // stage the next tile before this tile's first output store: the wait on the
            // prefetch loads then never includes stores
            if (f == 0 && tn >= 0) st.store(s[cur ^ 1]);
            if constexpr (SSE) sse_block(gy ? gy + plane : nullptr, y ? y + plane : nullptr, W, H, x0, y0, vec, acc, tv, sq);
            else store_block(y + plane, W, H, x0, y0, vec, acc);
        }
        __syncthreads();
        cur ^= 1;
        t = tn;
    }
    if constexpr (SSE) block_sum_store(sq, reinterpret_cast<double*>(&s[0][0]), part);
}

// Three waves per SIMD (the x tiles' LDS allows three work-groups per CU): the plain
// forward fits without the hint; the fused forward with late target loads fits with it.
template <int R, bool SSE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void bank_fwd_pers_k(
    const float* __restrict__ x, const float* __restrict__ w, float* __restrict__ y, const float* __restrict__ tg,
    float* __restrict__ gy, double* __restrict__ part, int F, int H, int W, int tiles_x, int tiles_img, int ntiles,
    int vec) {
    bank_fwd_pers_body<R, SSE, false>(x, w, y, tg, gy, part, F, H, W, tiles_x, tiles_img, ntiles, vec);
}

// Fused forward with the target block loaded before the FMAs: more live registers, two waves.
template <int R>
__global__ __launch_bounds__(256) void bank_fwd_sse_tpre_k(const float* __restrict__ x, const float* __restrict__ w,
                                                           float* __restrict__ y, const float* __restrict__ tg,
                                                           float* __restrict__ gy, double* __restrict__ part, int F,
                                                           int H, int W, int tiles_x, int tiles_img, int ntiles,
                                                           int vec) {
    bank_fwd_pers_body<R, true, true>(x, w, y, tg, gy, part, F, H, W, tiles_x, tiles_img, ntiles, vec);
}

template <int R>
__global__ __launch_bounds__(256) void bank_bwd_in_pers_k(const float* __restrict__ gy, const float* __restrict__ w,
                                                          float* __restrict__ gx, int F, int H, int W, int tiles_x,
                                                          int tiles_img, int ntiles, int vec,
                                                          const float* __restrict__ scale) {
    using G = BankTile<R>;
    constexpr int LW = G::LW, NR = G::NR, RA = G::RA, N = 2 * R + 1, NP = (N + 3) & ~3;
    __shared__ __attribute__((aligned(16))) float s[NR * LW];
    __shared__ __attribute__((aligned(16))) float wl[PERS_FMAX * N * NP];
    taps_to_lds<R, true>(w, F, wl);
    const size_t hw = (size_t)H * W;
    Stage<F32, NR, LW, true> st;   // zero outside the image: gy is extended by zero
    auto fetch = [&](int t, int f) {
        const int n = t / tiles_img, ti = t - n * tiles_img;
        int x0, y0;
        tile_origin(ti, tiles_x, BT, BT, x0, y0);
        st.load(gy + ((size_t)n * F + f) * hw, (size_t)W * 4, W, H, x0 - RA, y0 - R, vec);
    };
    const BandWalk walk(tiles_x, ntiles / tiles_x);   // images stacked vertically
    int t = walk.tile(0);
    if (t >= 0) fetch(t, 0);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int k = 0; t >= 0; t = walk.tile(++k)) {
        const int tnext = walk.tile(k + 1);
        const int n = t / tiles_img, ti = t - n * tiles_img;
        int x0, y0;
        tile_origin(ti, tiles_x, BT, BT, x0, y0);
        float acc[BPY][BPX] = {};
#pragma unroll 1
        for (int f = 0; f < F; ++f) {
            st.store(s);
            __syncthreads();
            const int nt = (f + 1 < F) ? t : tnext;
            if (nt >= 0) fetch(nt, (f + 1 < F) ? f + 1 : 0);
            corr_rows<R, BPX, BPY, LW, true>(&s[(ty * BPY) * LW + tx * BPX], &wl[f * N * NP], acc);
            __syncthreads();
        }
        scale_acc(acc, out_scale(scale));
        store_block(gx + (size_t)n * hw, W, H, x0, y0, vec, acc);
    }
}

// Filter gradient, four filters per 256-lane block: the x tile (64x64 pixels plus halo)
// is staged once and shared by the four waves; wave w accumulates all taps of filter
// 4*group + w over the tile's 4096 pixels (lane = column, 64 rows), then reduces over
// the wave and writes one partial per tap.
constexpr int GW4_T = 64;

// TY 64-row sub-tiles per work-group: the wave's (2r+1)^2 accumulators run over all of them
// before the one cross-lane reduction, so TY > 1 divides that reduction and the partials.
template <int R, int TY, int CH = GW_CH>
__global__ __launch_bounds__(256) void bank_bwd_w4_k(const float* __restrict__ gy, const float* __restrict__ x,
                                                     float* __restrict__ part, int F, int H, int W, int tiles_x,
                                                     int tiles_img, int ntiles, int fgroups) {
    constexpr int N = 2 * R + 1, RA = (R + 3) & ~3, LW = GW4_T + 2 * RA, NR = GW4_T + 2 * R;
    __shared__ __attribute__((aligned(16))) float s[NR * LW];
    const unsigned id = xcd_remap(blockIdx.x, gridDim.x);
    const int fg = (int)(id % (unsigned)fgroups);
    const int tile = (int)(id / (unsigned)fgroups);
    const int n = tile / tiles_img, ti = tile - n * tiles_img;
    int x0, y0;
    tile_origin(ti, tiles_x, GW4_T, GW4_T * TY, x0, y0);
    const size_t hw = (size_t)H * W;
    const float* xp = x + (size_t)n * hw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f = fg * 4 + wave;
    const bool live = f < F;   // a wave past the last filter still joins the barriers
    const float* g = gy + ((size_t)n * F + (live ? f : 0)) * hw;
    const int gxp = x0 + lane;
    float acc[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) acc[j][i] = 0.f;
    for (int sub = 0; sub < TY; ++sub) {
        const int ys = y0 + sub * GW4_T;
        if (ys >= H) break;   // uniform over the work-group
        if (sub) __syncthreads();   // the previous sub-tile is consumed
        if constexpr (TY == 1) {
            stage_clamped<NR, LW>(xp, W, H, x0 - RA, ys - R, s);
        } else {   // accumulators live across the sub-tiles leave no registers for a batch of loads
            for (int idx = threadIdx.x; idx < NR * LW; idx += 256) {
                const int rr = idx / LW, c = idx - rr * LW;
                s[idx] = xp[(size_t)clampi(ys - R + rr, H) * W + clampi(x0 - RA + c, W)];
            }
        }
        __syncthreads();
        if (!live) continue;
#pragma unroll 1
        for (int r0 = 0; r0 < GW4_T; r0 += CH) {
            float gv[CH];
#pragma unroll
            for (int py = 0; py < CH; ++py) {
                const int yy = ys + r0 + py;
                gv[py] = (gxp < W && yy < H) ? g[(size_t)yy * W + gxp] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                float cv[CH + 2 * R];
#pragma unroll
                for (int m = 0; m < CH + 2 * R; ++m) cv[m] = s[(r0 + m) * LW + lane + RA - R + i];
#pragma unroll
                for (int j = 0; j < N; ++j)
#pragma unroll
                    for (int py = 0; py < CH; ++py) acc[j][i] = fmaf(gv[py], cv[py + j], acc[j][i]);
            }
        }
    }
    if (!live) return;
    float* out = part + (size_t)f * N * N * ntiles + tile;
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float v = acc[j][i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) out[(size_t)(j * N + i) * ntiles] = v;
        }
}

// ------------------------------------------------------------------ filter gradient on the matrix cores
// gw[f][k] = sum_p gy[f][p] x[p + off(k)] is a matrix product: filters as rows, taps as
// columns, pixels as the reduction.  v_mfma_f32_16x16x4f32 takes four pixels per step:
//   A[f][q] = gy[f][p_q]           lane f + 16q
//   B[q][j] = x[p_q + off(16t + j)] lane j + 16q      (tap column block t of ceil(NK/16))
//   D[f][j] += sum_q A[f][q] B[q][j] lane j + 16(f/4), register f % 4
// Each work-group stages a 64-column x 64-row x tile (with halo, clamped) in LDS; its four
// waves take 16 rows each, every row as 16 four-pixel steps, the 16 x 4 gy values of a row
// loaded ahead in registers.  The four waves' sums are added in a fixed order and written as
// one partial per (filter, tap, tile), so the result is deterministic.  Up to 16 filters.
constexpr int GWM_T = 64;

// The staged rows are LWS = 64 + 2 RA pixels at a stride of LWS + 8 floats: a row stride of
// 16 words modulo 64 puts the taps of one 16-tap block, which span up to three window rows, in
// distinct LDS banks.  The cross-wave reduction reuses the tile's LDS once the products are
// done, so a work-group holds one buffer (about 24 KB at r = 4: six work-groups per CU).
// PX: step st of a row takes pixels st, 16 + st, 32 + st, 48 + st (k = pixel / 16) instead of
// 4 st .. 4 st + 3, so each lane's 16 gy values of a row are 16 consecutive pixels, read as four
// 16-byte vectors; the products are the same, summed in another order.
// TAIL (for (2r+1)^2 = 1 mod 16, r = 3 and 4): the last tap, alone in its 16-tap block, is summed
// by each lane with vector FMAs after each row's products (its own gy times the row's x at that
// tap, four 16-byte LDS reads where aligned) instead of a block of matrix products that is 15/16
// padding, and its four pixel groups are added with two cross-lane shuffles.  At four waves per
// SIMD the edge strips' per-step column offsets go to scratch (52 bytes per lane at r = 4,
// reloaded only on the scalar edge path).
template <int R, int TY, bool PX = false, bool TAIL = false>
__global__ __launch_bounds__(256, 4) void bank_bwd_wm_k(const float* __restrict__ gy, const float* __restrict__ x,
                                                     float* __restrict__ part, int F, int H, int W, int tiles_x,
                                                     int tiles_img, int ntiles) {
    constexpr int N = 2 * R + 1, NK = N * N, NT = (NK + 15) / 16;
    constexpr bool TV = TAIL && NK % 16 == 1;
    constexpr int NTM = TV ? NT - 1 : NT;   // 16-tap blocks on the matrix cores
    constexpr int RA = (R + 3) & ~3, LWS = GWM_T + 2 * RA, LW = LWS + 8, NR = GWM_T + 2 * R;
    constexpr int S_FLOATS = NR * LW, RED_FLOATS = 4 * 16 * NT * 16;
    __shared__ __attribute__((aligned(16))) float s[S_FLOATS > RED_FLOATS ? S_FLOATS : RED_FLOATS];
    auto red = reinterpret_cast<float (*)[16][NT * 16]>(s);
    const unsigned id = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)id;
    const int n = tile / tiles_img, ti = tile - n * tiles_img;
    int x0, y0;
    tile_origin(ti, tiles_x, GWM_T, GWM_T * TY, x0, y0);
    const size_t hw = (size_t)H * W;
    const float* xp = x + (size_t)n * hw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int fl = lane & 15, q = lane >> 4;   // A row (filter) / B column (tap in block); pixel of the step
    const bool frow = fl < F;
    const float* g = gy + ((size_t)n * F + (frow ? fl : 0)) * hw;
    int off[NT];   // LDS offset of this lane's tap (clamped into range for the padding columns)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int k = min(16 * t + fl, NK - 1);
        off[t] = (k / N) * LW + (k % N) + RA - R;
    }
    v4f acc[NTM];
#pragma unroll
    for (int t = 0; t < NTM; ++t) acc[t] = mk4(0.f, 0.f, 0.f, 0.f);
    constexpr int OFFL = ((NK - 1) / N) * LW + (NK - 1) % N + RA - R;   // the last tap's LDS offset
    float accl = 0.f;
    // a row's 16 x 4 gy values; pixels outside the image (and filters past F) contribute 0.
    // The load itself always reads a valid (clamped) address, so no lane branches around it.
    const bool vec = (W & 3) == 0 && ((uintptr_t)gy & 15) == 0;
    auto gy_row = [&](int yy, float (&ga)[16]) {
        const float* grow = g + (size_t)min(yy, H - 1) * W;
        if constexpr (PX) {
            const int xb = x0 + 16 * q;
            if (vec && xb + 16 <= W) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const v4f v = *reinterpret_cast<const v4f*>(grow + xb + 4 * m);
#pragma unroll
                    for (int e = 0; e < 4; ++e) ga[4 * m + e] = (frow && yy < H) ? v[e] : 0.f;
                }
            } else {
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const int xx = xb + st;
                    const float v = grow[min(xx, W - 1)];
                    ga[st] = (frow && xx < W && yy < H) ? v : 0.f;
                }
            }
            return;
        }
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int xx = x0 + 4 * st + q;
            const float v = grow[min(xx, W - 1)];
            ga[st] = (frow && xx < W && yy < H) ? v : 0.f;
        }
    };
    // LDS column of step st's pixel for this lane
    auto pcol = [&](int st) { return PX ? 16 * q + st : 4 * st + q; };
    // the last tap over a row's 16 steps: with pixel-strided steps its 16 x values are
    // consecutive, read as four 16-byte vectors where the offset allows
    auto tail = [&](int py, const float (&g)[16]) {
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (PX && (LW % 4 == 0) && (OFFL % 4 == 0)) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const v4f v = lds4(&s[py * LW + 16 * q + OFFL + 4 * m]);
#pragma unroll
                for (int e = 0; e < 4; ++e) accl = fmaf(g[4 * m + e], v[e], accl);
            }
        } else {
#pragma unroll
            for (int st = 0; st < 16; ++st) accl = fmaf(g[st], s[py * LW + pcol(st) + OFFL], accl);
        }
    };
    for (int sub = 0; sub < TY; ++sub) {
        const int ys = y0 + sub * GWM_T;
        if (ys >= H) break;   // uniform over the work-group
        if (sub) __syncthreads();
        if constexpr (TY == 1) {
            stage_clamped<NR, LW, LWS>(xp, W, H, x0 - RA, ys - R, s);
        } else {   // accumulators live across the sub-tiles leave no registers for a batch of loads
            for (int idx = threadIdx.x; idx < NR * LWS; idx += 256) {
                const int rr = idx / LWS, c = idx - rr * LWS;
                s[rr * LW + c] = xp[(size_t)clampi(ys - R + rr, H) * W + clampi(x0 - RA + c, W)];
            }
        }
        __syncthreads();
        float ga[16], gb[16];
        gy_row(ys + wave * 16, ga);
#pragma unroll 1
        for (int row = 0; row < 16; row += 2) {
            const int py = wave * 16 + row;
            gy_row(ys + py + 1, gb);   // the next row's gy in flight during this row's products
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int base = py * LW + pcol(st);
#pragma unroll
                for (int t = 0; t < NTM; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[st], s[base + off[t]], acc[t], 0, 0, 0);
            }
            if constexpr (TV) tail(py, ga);
            if (row + 2 < 16) gy_row(ys + py + 2, ga);
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int base = (py + 1) * LW + pcol(st);
#pragma unroll
                for (int t = 0; t < NTM; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gb[st], s[base + off[t]], acc[t], 0, 0, 0);
            }
            if constexpr (TV) tail(py + 1, gb);
        }
    }
    // lane holds D[4 (lane / 16) + i][16 t + lane % 16] in acc[t][i]; the tile's products are
    // done (the barrier) before its LDS takes the partial sums
    if constexpr (TV) {   // lane (filter fl, pixel group q): add the four pixel groups
        accl += __shfl_xor(accl, 16, 64);
        accl += __shfl_xor(accl, 32, 64);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave][4 * q + i][16 * t + fl] = acc[t][i];
    if constexpr (TV)
        if (q == 0) red[wave][fl][NK - 1] = accl;
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * NK; e += 256) {
        const int f = e / NK, k = e - f * NK;
        if (f >= F) continue;
        const float v = ((red[0][f][k] + red[1][f][k]) + red[2][f][k]) + red[3][f][k];
        part[((size_t)f * NK + k) * ntiles + tile] = v;
    }
}

template <int R, int TY, bool PX = false, bool TAIL = false>
hipError_t bwd_wm_RT(const BankArgs& a) {
    const int tx = (a.w + GWM_T - 1) / GWM_T, ty = (a.h + GWM_T * TY - 1) / (GWM_T * TY);
    const int ntiles = a.n * tx * ty;
    float* part = static_cast<float*>(a.ws);
    hipLaunchKernelGGL((bank_bwd_wm_k<R, TY, PX, TAIL>), dim3((unsigned)ntiles), dim3(256), 0, a.st, a.a, a.b, part, a.f, a.h,
                       a.w, tx, tx * ty, ntiles);
    const int nk = (2 * R + 1) * (2 * R + 1);
    hipLaunchKernelGGL(bank_bwd_w2_k, dim3((unsigned)(a.f * nk)), dim3(256), 0, a.st, part, a.out, ntiles, a.scale);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
int bank_vec(const float* a, const float* b, int W) {
    return ((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0) && (W % 4 == 0);
}

template <int R>
hipError_t fwd_R(const BankArgs& a) {
    const int tx = (a.w + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    hipLaunchKernelGGL(bank_fwd_k<R>, dim3((unsigned)(a.n * tx * ty)), dim3(256), 0, a.st, a.a, a.b, a.out, a.f, a.h,
                       a.w, tx, tx * ty, bank_vec(a.a, a.out, a.w));
    return hipGetLastError();
}

template <int R>
hipError_t bwd_in_R(const BankArgs& a) {
    const int tx = (a.w + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    hipLaunchKernelGGL(bank_bwd_in_k<R>, dim3((unsigned)(a.n * tx * ty)), dim3(256), 0, a.st, a.a, a.b, a.out, a.f,
                       a.h, a.w, tx, tx * ty, bank_vec(a.a, a.out, a.w), a.scale);
    return launch_edge<R>(a);
}

template <int R>
hipError_t bwd_w_R(const BankArgs& a) {
    const int tx = (a.w + GW_TW - 1) / GW_TW, ty = (a.h + GW_TH - 1) / GW_TH;
    const int ntiles = a.n * tx * ty;
    float* part = static_cast<float*>(a.ws);
    hipLaunchKernelGGL(bank_bwd_w1_k<R>, dim3((unsigned)(ntiles * a.f)), dim3(64), 0, a.st, a.a, a.b, part, a.f, a.h,
                       a.w, tx, tx * ty, ntiles);
    const int nk = (2 * R + 1) * (2 * R + 1);
    hipLaunchKernelGGL(bank_bwd_w2_k, dim3((unsigned)(a.f * nk)), dim3(256), 0, a.st, part, a.out, ntiles, a.scale);
    return hipGetLastError();
}

hipError_t launch_fwd_plain(const BankArgs& a) {
    const long long tot = (long long)a.n * a.f * a.h * a.w;
    hipLaunchKernelGGL(bank_fwd_plain_k, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, a.st, a.a, a.b, a.out, a.n,
                       a.f, a.h, a.w, a.r);
    return hipGetLastError();
}

hipError_t launch_bwd_in_plain(const BankArgs& a) {
    const long long tot = (long long)a.n * a.h * a.w;
    hipLaunchKernelGGL(bank_bwd_in_plain_k, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, a.st, a.a, a.b, a.out,
                       a.n, a.f, a.h, a.w, a.r, a.scale);
    return hipGetLastError();
}

template <int R>
hipError_t fwd_pers_R(const BankArgs& a) {
    const int tx = (a.w + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    const int ntiles = a.n * tx * ty;
    const void* k = reinterpret_cast<const void*>(&bank_fwd_pers_k<R, false>);
    hipLaunchKernelGGL((bank_fwd_pers_k<R, false>), dim3(persistent_grid(k, 256, ntiles)), dim3(256), 0, a.st, a.a,
                       a.b, a.out, nullptr, nullptr, nullptr, a.f, a.h, a.w, tx, tx * ty, ntiles,
                       bank_vec(a.a, a.out, a.w));
    return hipGetLastError();
}

template <int R>
hipError_t bwd_in_pers_R(const BankArgs& a) {
    const int tx = (a.w + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    const int ntiles = a.n * tx * ty;
    const void* k = reinterpret_cast<const void*>(&bank_bwd_in_pers_k<R>);
    hipLaunchKernelGGL(bank_bwd_in_pers_k<R>, dim3(persistent_grid(k, 256, ntiles)), dim3(256), 0, a.st, a.a, a.b,
                       a.out, a.f, a.h, a.w, tx, tx * ty, ntiles, bank_vec(a.a, a.out, a.w), a.scale);
    return launch_edge<R>(a);
}

template <int R, int TY, int CH = GW_CH>
hipError_t bwd_w4_RT(const BankArgs& a) {
    const int tx = (a.w + GW4_T - 1) / GW4_T, ty = (a.h + GW4_T * TY - 1) / (GW4_T * TY);
    const int ntiles = a.n * tx * ty;
    const int fgroups = (a.f + 3) / 4;
    float* part = static_cast<float*>(a.ws);
    hipLaunchKernelGGL((bank_bwd_w4_k<R, TY, CH>), dim3((unsigned)(ntiles * fgroups)), dim3(256), 0, a.st, a.a, a.b,
                       part, a.f, a.h, a.w, tx, tx * ty, ntiles, fgroups);
    const int nk = (2 * R + 1) * (2 * R + 1);
    hipLaunchKernelGGL(bank_bwd_w2_k, dim3((unsigned)(a.f * nk)), dim3(256), 0, a.st, part, a.out, ntiles, a.scale);
    return hipGetLastError();
}

#define ICL_BANK_SWITCH(FN)                   \
    switch (a.r) {                            \
        case 1: return FN<1>(a);              \
        case 2: return FN<2>(a);              \
        case 3: return FN<3>(a);              \
        case 4: return FN<4>(a);              \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_fwd(const BankArgs& a) { ICL_BANK_SWITCH(fwd_R) }
hipError_t launch_bwd_in(const BankArgs& a) { ICL_BANK_SWITCH(bwd_in_R) }
hipError_t launch_bwd_w(const BankArgs& a) { ICL_BANK_SWITCH(bwd_w_R) }
hipError_t launch_fwd_pers(const BankArgs& a) { ICL_BANK_SWITCH(fwd_pers_R) }
hipError_t launch_bwd_in_pers(const BankArgs& a) { ICL_BANK_SWITCH(bwd_in_pers_R) }
template <int R>
hipError_t bwd_w4_R(const BankArgs& a) { return bwd_w4_RT<R, 1>(a); }
template <int R>
hipError_t bwd_w4x4_R(const BankArgs& a) { return bwd_w4_RT<R, 4>(a); }

template <int R>
hipError_t bwd_wm_R(const BankArgs& a) { return bwd_wm_RT<R, 1>(a); }
template <int R>
hipError_t bwd_wm4_R(const BankArgs& a) { return bwd_wm_RT<R, 4>(a); }
template <int R>
hipError_t bwd_wmp_R(const BankArgs& a) { return bwd_wm_RT<R, 1, true>(a); }
template <int R>
hipError_t bwd_wmp4_R(const BankArgs& a) { return bwd_wm_RT<R, 4, true>(a); }
template <int R>
hipError_t bwd_wmpt4_R(const BankArgs& a) { return bwd_wm_RT<R, 4, true, true>(a); }

hipError_t launch_bwd_w4(const BankArgs& a) { ICL_BANK_SWITCH(bwd_w4_R) }
hipError_t launch_bwd_wm(const BankArgs& a) { ICL_BANK_SWITCH(bwd_wm_R) }
hipError_t launch_bwd_wm4(const BankArgs& a) { ICL_BANK_SWITCH(bwd_wm4_R) }
hipError_t launch_bwd_wmp(const BankArgs& a) { ICL_BANK_SWITCH(bwd_wmp_R) }
hipError_t launch_bwd_wmp4(const BankArgs& a) { ICL_BANK_SWITCH(bwd_wmp4_R) }
hipError_t launch_bwd_wmpt4(const BankArgs& a) { ICL_BANK_SWITCH(bwd_wmpt4_R) }
hipError_t launch_bwd_w4x4(const BankArgs& a) { ICL_BANK_SWITCH(bwd_w4x4_R) }


bool supports_bank(const BankArgs& a) { return a.r >= 1 && a.r <= 4 && a.f >= 1 && a.f <= 64; }
bool supports_pers(const BankArgs& a) { return supports_bank(a) && a.f <= PERS_FMAX; }
bool supports_bwd_w(const BankArgs& a) {
    return supports_bank(a) && a.ws != nullptr && a.wsb >= bank_bwd_filter_workspace(a.n, a.f, a.h, a.w, a.r);
}
bool supports_bwd_wm(const BankArgs& a) { return supports_bwd_w(a) && a.f <= 16; }


const Variant<BankArgs> kBwdIn[] = {{"plain", supports_bank, launch_bwd_in_plain},
                                    {"tile64_p4x4_fold", supports_bank, launch_bwd_in},
                                    {"pers_p4x4_fold", supports_pers, launch_bwd_in_pers}};
const Variant<BankArgs> kBwdW[] = {{"wave_t32x64", supports_bwd_w, launch_bwd_w},
                                   {"block4_t64", supports_bwd_w, launch_bwd_w4},
                                   {"block4_t64x256", supports_bwd_w, launch_bwd_w4x4},
                                   {"mfma_t64", supports_bwd_wm, launch_bwd_wm},
                                   {"mfma_t64x256", supports_bwd_wm, launch_bwd_wm4},
                                   {"mfma_px_t64", supports_bwd_wm, launch_bwd_wmp},
                                   {"mfma_px_t64x256", supports_bwd_wm, launch_bwd_wmp4},
                                   {"mfma_px_tail_t64x256", supports_bwd_wm, launch_bwd_wmpt4}};

// ------------------------------------------------------------------ forward on the matrix cores
// y[f][p] = sum_k w[f][k] x[p + off(k)]: filters as rows, pixels as columns, taps as the
// reduction, in v_mfma_f32_16x16x4f32 steps of four taps:
//   A[f][k] = w[f][4s + k]          lane f + 16k  (zero past the last tap or filter)
//   B[k][j] = x[p_j + off(4s + k)]  lane j + 16k  (16 consecutive pixels of a tile row)
//   D[f][j]                         lane j + 16(f/4), register f % 4
// A persistent grid walks 64 x 64 tiles; each is staged in LDS (clamped) and its four waves
// take 16 rows each, four 16-pixel column groups at a time (four independent accumulator
// chains).  SSE: the loss epilogue of the fused forward (gy = 2 (y - t), y on request, the
// work-group's double partial of sum (y - t)^2).  Up to 16 filters.
// WAVES > 0: the register budget of WAVES waves per SIMD (the LDS tile admits more work-groups
// than the unconstrained allocation leaves room for).
// PX: the operands swap roles (pixels as rows, filters as columns), which changes nothing in
// the products or their order but puts four consecutive pixels of one filter in each lane's
// accumulator, so the targets are read and the outputs written as 16-byte vectors (a quarter
// of the memory instructions of the filter-major layout, where a lane holds one pixel of four
// filters).
template <int R, bool SSE, int WAVES = 0, bool PX = false>
__global__ __launch_bounds__(256, WAVES > 0 ? WAVES : 1) void bank_fwd_mfma_k(const float* __restrict__ x,
                                                                             const float* __restrict__ w,
                                                       float* __restrict__ y, const float* __restrict__ tg,
                                                       float* __restrict__ gy, double* __restrict__ part, int F,
                                                       int H, int W, int tiles_x, int tiles_img, int ntiles, int vec) {
    using G = BankTile<R>;
    constexpr int N = 2 * R + 1, NK = N * N, NS = (NK + 3) / 4;
    constexpr int LW = G::LW, NR = G::NR, RA = G::RA;
    __shared__ __attribute__((aligned(16))) float s[NR * LW];
    __shared__ double red[256];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, kq = lane >> 4;
    float a[NS];
    int off[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
        const int k = 4 * st + kq;
        a[st] = (k < NK && j < F) ? w[j * NK + k] : 0.f;
        const int kc = k < NK ? k : NK - 1;   // padding taps read a valid pixel, times zero
        off[st] = (kc / N) * LW + (kc % N) + RA - R;
    }
    const size_t hw = (size_t)H * W;
    double sq = 0.0;
    for (int t = (int)blockIdx.x; t < ntiles; t += (int)gridDim.x) {
        const int n = t / tiles_img, ti = t - n * tiles_img;
        int x0, y0;
        tile_origin(ti, tiles_x, BT, BT, x0, y0);
        __syncthreads();   // the previous tile's products are done with s
        stage_plane<R, false>(x + (size_t)n * hw, W, H, x0, y0, vec, s);
        __syncthreads();
        if constexpr (PX) {
            // lane: filter j, pixels 16 c + 4 kq + (0..3) of the row, c = 0..3
            const int fj = min(j, F - 1);
            const float* tplane = SSE ? tg + ((size_t)n * F + fj) * hw : nullptr;
#pragma unroll 1
            for (int row = 0; row < 16; ++row) {
                const int py = wave * 16 + row;
                const int yg = y0 + py;
                const size_t rowoff = (size_t)min(yg, H - 1) * W;
                v4f tv[4];
                if constexpr (SSE) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int xg = x0 + 16 * c + 4 * kq;
                        if (vec && xg + 4 <= W) {
                            tv[c] = *reinterpret_cast<const v4f*>(tplane + rowoff + xg);
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i) tv[c][i] = tplane[rowoff + min(xg + i, W - 1)];
                        }
                    }
                }
                v4f acc[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = mk4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int st = 0; st < NS; ++st)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(s[py * LW + 16 * c + j + off[st]], a[st], acc[c],
                                                                      0, 0, 0);
                if (yg >= H || j >= F) continue;
                float ssum = 0.f;
                const size_t plane = ((size_t)n * F + j) * hw + (size_t)yg * W;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int xg = x0 + 16 * c + 4 * kq;
                    if (xg >= W) continue;
                    const bool full = vec && xg + 4 <= W;
                    if constexpr (SSE) {
                        v4f d = acc[c] - tv[c];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (full || xg + i < W) ssum = fmaf(d[i], d[i], ssum);
                        const v4f g2 = 2.f * d;
                        if (full) {
                            if (gy) *reinterpret_cast<v4f*>(gy + plane + xg) = g2;
                            if (y) *reinterpret_cast<v4f*>(y + plane + xg) = acc[c];
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                if (xg + i >= W) break;
                                if (gy) gy[plane + xg + i] = g2[i];
                                if (y) y[plane + xg + i] = acc[c][i];
                            }
                        }
                    } else {
                        if (full) {
                            *reinterpret_cast<v4f*>(y + plane + xg) = acc[c];
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (xg + i < W) y[plane + xg + i] = acc[c][i];
                        }
                    }
                }
                if constexpr (SSE) sq += (double)ssum;
            }
            continue;
        }
#pragma unroll 1
        for (int row = 0; row < 16; ++row) {
            const int py = wave * 16 + row;
            const int yg = y0 + py;
            // the lane's 4 x 4 targets, loaded before the products so that their latency hides
            // under the matrix work (a valid clamped address, zero weight outside the image)
            float tv[4][4];
            if constexpr (SSE) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int f = min(4 * kq + i, F - 1);
                        const int xg = min(x0 + 16 * c + j, W - 1);
                        tv[c][i] = tg[((size_t)n * F + f) * hw + (size_t)min(yg, H - 1) * W + xg];
                    }
            }
            v4f acc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = mk4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], s[py * LW + 16 * c + j + off[st]], acc[c],
                                                                  0, 0, 0);
            if (yg >= H) continue;
            float ssum = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int xg = x0 + 16 * c + j;
                if (xg >= W) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int f = 4 * kq + i;
                    if (f >= F) continue;
                    const size_t q = ((size_t)n * F + f) * hw + (size_t)yg * W + xg;
                    if constexpr (SSE) {
                        const float d = acc[c][i] - tv[c][i];
                        ssum = fmaf(d, d, ssum);
                        if (gy) gy[q] = 2.f * d;
                        if (y) y[q] = acc[c][i];
                    } else {
                        y[q] = acc[c][i];
                    }
                }
            }
            if constexpr (SSE) sq += (double)ssum;
        }
    }
    if constexpr (SSE) block_sum_store(sq, red, part);
}

template <int R, bool PX = false>
hipError_t fwd_mfma_R(const BankArgs& a) {
    const int tx = (a.w + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    const int ntiles = a.n * tx * ty;
    const void* k = reinterpret_cast<const void*>(&bank_fwd_mfma_k<R, false, 0, PX>);
    hipLaunchKernelGGL((bank_fwd_mfma_k<R, false, 0, PX>), dim3(persistent_grid(k, 256, ntiles)), dim3(256), 0, a.st,
                       a.a, a.b, a.out, nullptr, nullptr, nullptr, a.f, a.h, a.w, tx, tx * ty, ntiles,
                       bank_vec(a.a, a.out, a.w));
    return hipGetLastError();
}
template <int R>
hipError_t fwd_mfma_px_R(const BankArgs& a) { return fwd_mfma_R<R, true>(a); }

hipError_t launch_fwd_mfma(const BankArgs& a) { ICL_BANK_SWITCH(fwd_mfma_R) }
hipError_t launch_fwd_mfma_px(const BankArgs& a) { ICL_BANK_SWITCH(fwd_mfma_px_R) }
bool supports_mfma16(const BankArgs& a) { return supports_bank(a) && a.f <= 16; }

const Variant<BankArgs> kFwd[] = {{"plain", supports_bank, launch_fwd_plain},
                                   {"tile64_p4x4", supports_bank, launch_fwd},
                                   {"pers_p4x4", supports_pers, launch_fwd_pers},
                                   {"mfma_t64", supports_mfma16, launch_fwd_mfma},
                                   {"mfma_px_t64", supports_mfma16, launch_fwd_mfma_px}};
// ------------------------------------------------------------------ sum of squares loss
constexpr int SSE_BLOCKS = 2048;

__global__ __launch_bounds__(256) void sse_k1(const float* __restrict__ y, const float* __restrict__ t,
                                              float* __restrict__ gy, long long count, float* __restrict__ part,
                                              int vec) {
    __shared__ float red[256];
    float acc = 0.f;
    const long long stride = (long long)gridDim.x * 256;
    if (vec) {
        const long long n4 = count / 4;
        for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < n4; q += stride) {
            const v4f a = reinterpret_cast<const v4f*>(y)[q];
            const v4f b = reinterpret_cast<const v4f*>(t)[q];
            const v4f d = a - b;
            acc = fmaf(d.x, d.x, acc); acc = fmaf(d.y, d.y, acc);
            acc = fmaf(d.z, d.z, acc); acc = fmaf(d.w, d.w, acc);
            if (gy) reinterpret_cast<v4f*>(gy)[q] = 2.f * d;
        }
        for (long long q = n4 * 4 + (long long)blockIdx.x * 256 + threadIdx.x; q < count; q += stride) {
            const float d = y[q] - t[q];
            acc = fmaf(d, d, acc);
            if (gy) gy[q] = 2.f * d;
        }
    } else {
        for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < count; q += stride) {
            const float d = y[q] - t[q];
            acc = fmaf(d, d, acc);
            if (gy) gy[q] = 2.f * d;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sse_k2(const float* __restrict__ part, int nparts, float* __restrict__ loss) {
    __shared__ float red[256];
    float v = 0.f;
    for (int q = threadIdx.x; q < nparts; q += 256) v += part[q];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

// ------------------------------------------------------------------ forward fused with the loss

// Plain fused forward: grid-stride over the outputs, each from its clamped taps directly
// (the same tap order as every FMA forward variant), double partial per work-group.
__global__ __launch_bounds__(256) void bank_fwd_sse_plain_k(const float* __restrict__ x, const float* __restrict__ w,
                                                            const float* __restrict__ tg, float* __restrict__ y,
                                                            float* __restrict__ gy, double* __restrict__ part, int N,
                                                            int F, int H, int W, int r) {
    __shared__ double red[256];
    const long long hw = (long long)H * W, total = (long long)N * F * hw;
    const int nk = 2 * r + 1;
    double sq = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        const int n = (int)(i / (F * hw));
        const int f = (int)((i / hw) % F);
        const int p = (int)(i % hw), py = p / W, px = p - py * W;
        const float* xp = x + (size_t)n * hw;
        const float* wf = w + (size_t)f * nk * nk;
        float acc = 0.f;
        for (int j = -r; j <= r; ++j)
            for (int q = -r; q <= r; ++q)
                acc = fmaf(wf[(j + r) * nk + (q + r)], xp[(size_t)clampi(py + j, H) * W + clampi(px + q, W)], acc);
        const float d = acc - tg[i];
        sq = fma((double)d, (double)d, sq);
        if (gy) gy[i] = 2.f * d;
        if (y) y[i] = acc;
    }
    block_sum_store(sq, red, part);
}

// L = sum of the partials in a fixed order, in double, rounded once to float32.
__global__ __launch_bounds__(256) void sse_final_k(const double* __restrict__ part, int nparts, float* __restrict__ loss) {
    __shared__ double red[256];
    double v = 0.0;
    for (int q = threadIdx.x; q < nparts; q += 256) v += part[q];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)red[0];
}

int sse_vec(const BankSseArgs& a) {
    auto al = [](const void* p) { return p == nullptr || (uintptr_t)p % 16 == 0; };
    return al(a.x) && al(a.t) && al(a.y) && al(a.gy) && (a.wd % 4 == 0);
}

hipError_t launch_fwd_sse_plain(const BankSseArgs& a) {
    double* part = static_cast<double*>(a.ws);
    const long long tot = (long long)a.n * a.f * a.h * a.wd;
    const int grid = (int)std::min<long long>(FWD_SSE_PARTS, (tot + 255) / 256);
    hipLaunchKernelGGL(bank_fwd_sse_plain_k, dim3(grid), dim3(256), 0, a.st, a.x, a.w, a.t, a.y, a.gy, part, a.n, a.f,
                       a.h, a.wd, a.r);
    hipLaunchKernelGGL(sse_final_k, dim3(1), dim3(256), 0, a.st, part, grid, a.loss);
    return hipGetLastError();
}

template <int R, bool TPRE>
hipError_t fwd_sse_pers_R(const BankSseArgs& a) {
    double* part = static_cast<double*>(a.ws);
    const int tx = (a.wd + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    const int ntiles = a.n * tx * ty;
    auto kern = TPRE ? bank_fwd_sse_tpre_k<R> : bank_fwd_pers_k<R, true>;
    const int grid = std::min(persistent_grid(reinterpret_cast<const void*>(kern), 256, ntiles), FWD_SSE_PARTS);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, a.st, a.x, a.w, a.y, a.t, a.gy, part, a.f, a.h, a.wd, tx,
                       tx * ty, ntiles, sse_vec(a));
    hipLaunchKernelGGL(sse_final_k, dim3(1), dim3(256), 0, a.st, part, grid, a.loss);
    return hipGetLastError();
}

template <bool TPRE>
hipError_t launch_fwd_sse_pers(const BankSseArgs& a) {
    switch (a.r) {
        case 1: return fwd_sse_pers_R<1, TPRE>(a);
        case 2: return fwd_sse_pers_R<2, TPRE>(a);
        case 3: return fwd_sse_pers_R<3, TPRE>(a);
        case 4: return fwd_sse_pers_R<4, TPRE>(a);
        default: return hipErrorInvalidValue;
    }
}

bool supports_sse(const BankSseArgs& a) {
    return a.r >= 1 && a.r <= 4 && a.f >= 1 && a.f <= 64 && a.ws != nullptr && a.wsb >= bank_fwd_sse_workspace();
}
bool supports_sse_pers(const BankSseArgs& a) { return supports_sse(a) && a.f <= PERS_FMAX; }
bool supports_sse_mfma(const BankSseArgs& a) { return supports_sse(a) && a.f <= 16; }

template <int R, int WAVES = 0, bool PX = false>
hipError_t fwd_sse_mfma_R(const BankSseArgs& a) {
    double* part = static_cast<double*>(a.ws);
    const int tx = (a.wd + BT - 1) / BT, ty = (a.h + BT - 1) / BT;
    const int ntiles = a.n * tx * ty;
    const void* k = reinterpret_cast<const void*>(&bank_fwd_mfma_k<R, true, WAVES, PX>);
    const int grid = std::min(persistent_grid(k, 256, ntiles), FWD_SSE_PARTS);
    hipLaunchKernelGGL((bank_fwd_mfma_k<R, true, WAVES, PX>), dim3(grid), dim3(256), 0, a.st, a.x, a.w, a.y, a.t, a.gy, part, a.f,
                       a.h, a.wd, tx, tx * ty, ntiles, sse_vec(a));
    hipLaunchKernelGGL(sse_final_k, dim3(1), dim3(256), 0, a.st, part, grid, a.loss);
    return hipGetLastError();
}

template <int WAVES = 0, bool PX = false>
hipError_t launch_fwd_sse_mfma(const BankSseArgs& a) {
    switch (a.r) {
        case 1: return fwd_sse_mfma_R<1, WAVES, PX>(a);
        case 2: return fwd_sse_mfma_R<2, WAVES, PX>(a);
        case 3: return fwd_sse_mfma_R<3, WAVES, PX>(a);
        case 4: return fwd_sse_mfma_R<4, WAVES, PX>(a);
        default: return hipErrorInvalidValue;
    }
}

// pers_p4x4_tpre loads the lane's target block before the FMAs (more registers, fewer
// waves); pers_p4x4 loads it after them and relies on the other resident waves.
const Variant<BankSseArgs> kFwdSse[] = {{"plain", supports_sse, launch_fwd_sse_plain},
                                        {"pers_p4x4", supports_sse_pers, launch_fwd_sse_pers<false>},
                                        {"pers_p4x4_tpre", supports_sse_pers, launch_fwd_sse_pers<true>},
                                        {"mfma_t64", supports_sse_mfma, launch_fwd_sse_mfma<0>},
                                        {"mfma_t64_w4", supports_sse_mfma, launch_fwd_sse_mfma<4>},
                                        {"mfma_px_t64", supports_sse_mfma, launch_fwd_sse_mfma<0, true>}};

}  // namespace

size_t bank_bwd_filter_workspace(int n, int f, int h, int w, int r) {
    // partials of the variant with the most tiles (the 32x64 wave tiling)
    const size_t tx = (size_t)(w + GW_TW - 1) / GW_TW, ty = (size_t)(h + GW_TH - 1) / GW_TH;
    const size_t tx4 = (size_t)(w + GW4_T - 1) / GW4_T, ty4 = (size_t)(h + GW4_T - 1) / GW4_T;
    const size_t nk = (size_t)(2 * r + 1) * (2 * r + 1);
    const size_t tiles = tx * ty > tx4 * ty4 ? tx * ty : tx4 * ty4;
    return (size_t)n * tiles * (size_t)f * nk * sizeof(float);
}

size_t sse_workspace(long long) { return SSE_BLOCKS * sizeof(float); }

size_t bank_fwd_sse_workspace() { return FWD_SSE_PARTS * sizeof(double); }

namespace {
__global__ __launch_bounds__(256) void zero_k(float* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}
}  // namespace

hipError_t zero_fill(float* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t sse_launch(const float* y, const float* t, float* gy, long long count, float* loss, void* ws, size_t,
                      hipStream_t st) {
    float* part = static_cast<float*>(ws);
    const int vec = ((uintptr_t)y % 16 == 0) && ((uintptr_t)t % 16 == 0) && (gy == nullptr || (uintptr_t)gy % 16 == 0);
    hipLaunchKernelGGL(sse_k1, dim3(SSE_BLOCKS), dim3(256), 0, st, y, t, gy, count, part, vec);
    hipLaunchKernelGGL(sse_k2, dim3(1), dim3(256), 0, st, part, SSE_BLOCKS, loss);
    return hipGetLastError();
}

const Variant<BankArgs>* bank_fwd_variants(int* count) {
    *count = (int)(sizeof(kFwd) / sizeof(kFwd[0]));
    return kFwd;
}
const Variant<BankArgs>* bank_bwd_input_variants(int* count) {
    *count = (int)(sizeof(kBwdIn) / sizeof(kBwdIn[0]));
    return kBwdIn;
}
const Variant<BankArgs>* bank_bwd_filter_variants(int* count) {
    *count = (int)(sizeof(kBwdW) / sizeof(kBwdW[0]));
    return kBwdW;
}

int bank_fwd_default(const BankArgs& a) { return supports_mfma16(a) ? 4 : supports_pers(a) ? 2 : 1; }   // mfma_px_t64
int bank_bwd_input_default(const BankArgs& a) { return supports_pers(a) ? 2 : 1; }
int bank_bwd_filter_default(const BankArgs& a) { return a.f <= 16 ? 7 : 2; }   // mfma_px_tail_t64x256, else block4_t64x256
const Variant<BankSseArgs>* bank_fwd_sse_variants(int* count) {
    *count = (int)(sizeof(kFwdSse) / sizeof(kFwdSse[0]));
    return kFwdSse;
}
int bank_fwd_sse_default(const BankSseArgs& a) {   // mfma_px_t64, else pers_p4x4, else plain
    return supports_sse_mfma(a) ? 5 : supports_sse_pers(a) ? 1 : 0;
}

}  // namespace icl
