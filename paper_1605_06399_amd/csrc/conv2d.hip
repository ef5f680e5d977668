// Full 2-D correlation with clamped reads (ImageCL paper, Section 6:
// non-separable convolution benchmark, taps known only at run time, Table 3).
//
//   dst(x,y) = sum_{j,i=-r..r} w[(j+r)(2r+1) + (i+r)] * src(clamp(x+i), clamp(y+j))
//
// Variants
//   plain                 : one thread per pixel, 16x16 work-groups, clamp on every
//                           read, runtime loops, taps from global memory.
//   lds_p{PX}x{PY}_o{ORD} : a 16x16 work-group computes a 16*PX x 16*PY tile; the
//                           (TH+2r) x (TW+2*RA) input tile is staged once in LDS
//                           (float4 loads for interior tiles) and each lane keeps a
//                           PX x PY block of accumulators (thread coarsening,
//                           blocked mapping).  Taps are wave-uniform and live in
//                           SGPRs (the paper's constant-memory choice).
//                           ORD 0 walks tap rows outermost (one tap row of SGPRs
//                           live at a time, one LDS window per (tap row, output
//                           row)); ORD 1 walks staged input rows outermost (one LDS
//                           window per input row, every tap row it feeds).
//
// For r >= 3 the work is FP32-ALU bound on MI355X (2(2r+1)^2 flops per 8 bytes),
// so the variants aim at FMA density: no clamps in the inner loop, window reads
// as float4, taps as scalar operands.
#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "tile_stage.hpp"
#include "corr_tile.hpp"

namespace icl {
namespace {

template <class T>
__global__ __launch_bounds__(256) void conv2d_plain(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                    size_t dp, int W, int H, const float* __restrict__ w, int r,
                                                    Border bd) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    const int n = 2 * r + 1;
    float acc = 0.f;
    for (int j = -r; j <= r; ++j) {
        const bool yout = y + j < 0 || y + j >= H;
        const size_t row = (size_t)clampi(y + j, H) * sp;
        for (int i = -r; i <= r; ++i) {
            const bool out = bd.constant && (yout || x + i < 0 || x + i >= W);
            acc += w[(j + r) * n + (i + r)] *
                   (out ? bd.value : load_px<T>(src, row + (size_t)clampi(x + i, W) * T::size));
        }
    }
    store_px<T>(dst, (size_t)y * dp + (size_t)x * T::size, acc);
}

template <class T>
hipError_t launch_plain_T(const Conv2dArgs& a) {
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
    hipLaunchKernelGGL(conv2d_plain<T>, grid, dim3(256), 0, a.st, a.src, a.sp, a.dst, a.dp, a.W, a.H, a.taps, a.r,
                       a.bd);
    return hipGetLastError();
}

hipError_t launch_plain(const Conv2dArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_plain_T<F32>(a);
        case ICL_F16: return launch_plain_T<F16>(a);
        default: return launch_plain_T<BF16>(a);
    }
}

bool supports_plain(const Conv2dArgs& a) { return a.r >= 0 && a.r <= ICL_MAX_RADIUS; }

// ------------------------------------------------------------------ LDS-staged, register-blocked
template <int R, int PX, int PY> struct Tile2d {
    static constexpr int TW = 16 * PX, TH = 16 * PY;
    static constexpr int RA = (R + 3) & ~3;
    static constexpr int LW = TW + 2 * RA;
    static constexpr int NR = TH + 2 * R;
    static constexpr int WIN = PX + 2 * RA;      // floats per window read (multiple of 4)
};

template <class T, int R, int PX, int PY, int ORD>
__global__ __launch_bounds__(256) void conv2d_lds(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                  size_t dp, int W, int H, const float* __restrict__ w,
                                                  int tiles_x, int vec_ok, Border bd) {
    using G = Tile2d<R, PX, PY>;
    constexpr int TW = G::TW, TH = G::TH, RA = G::RA, LW = G::LW, NR = G::NR, WIN = G::WIN;
    constexpr int N = 2 * R + 1;
    __shared__ __attribute__((aligned(16))) float in_s[NR * LW];
    const int tid = threadIdx.x;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (int)(t % (unsigned)tiles_x) * TW;
    const int y0 = (int)(t / (unsigned)tiles_x) * TH;

    if (vec_ok && x0 - RA >= 0 && x0 + TW + RA <= W) {
        // all loads first (rows clamped), then the constant rows and the LDS writes: a
        // load-then-write loop would wait on each load in turn
        constexpr int C4 = LW / 4, NCH = NR * C4, PER = (NCH + 255) / 256;
        v4f v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            v[i] = load4<T>(src, (size_t)clampi(y0 - R + rr, H) * sp + (size_t)(x0 - RA + 4 * c4) * T::size);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int yy = y0 - R + rr;
            if (bd.constant && (yy < 0 || yy >= H)) v[i] = mk4(bd.value, bd.value, bd.value, bd.value);
            lds4(&in_s[rr * LW + 4 * c4], v[i]);
        }
    } else {
        for (int idx = tid; idx < NR * LW; idx += 256) {
            const int rr = idx / LW, c = idx - rr * LW;
            const int yy = y0 - R + rr, xx = x0 - RA + c;
            in_s[rr * LW + c] = (bd.constant && (yy < 0 || yy >= H || xx < 0 || xx >= W))
                                    ? bd.value
                                    : load_px<T>(src, (size_t)clampi(yy, H) * sp + (size_t)clampi(xx, W) * T::size);
        }
    }
    __syncthreads();

    const int tx = tid & 15, ty = tid >> 4;
    float acc[PY][PX];
#pragma unroll
    for (int py = 0; py < PY; ++py)
#pragma unroll
        for (int px = 0; px < PX; ++px) acc[py][px] = 0.f;

    const float* base = &in_s[(ty * PY) * LW + tx * PX];
    if constexpr (ORD == 0) {
        // tap row j outermost, kept a real loop so only one row of taps is live in SGPRs
#pragma unroll 1
        for (int j = 0; j < N; ++j) {
            const float* wj = w + j * N;
            const float* bj = base + j * LW;
#pragma unroll
            for (int py = 0; py < PY; ++py) {
                float win[WIN];
#pragma unroll
                for (int m = 0; m < WIN / 4; ++m) {
                    const v4f v = lds4(bj + py * LW + 4 * m);
                    win[4 * m] = v.x; win[4 * m + 1] = v.y; win[4 * m + 2] = v.z; win[4 * m + 3] = v.w;
                }
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const float c = wj[i];
#pragma unroll
                    for (int px = 0; px < PX; ++px) acc[py][px] = fmaf(c, win[RA - R + px + i], acc[py][px]);
                }
            }
        }
    } else {
        // staged input row q outermost: one window read per row, applied to every output
        // row it feeds (tap row j = q - py, a wave-uniform condition)
#pragma unroll 1
        for (int q = 0; q < PY + 2 * R; ++q) {
            float win[WIN];
#pragma unroll
            for (int m = 0; m < WIN / 4; ++m) {
                const v4f v = lds4(base + q * LW + 4 * m);
                win[4 * m] = v.x; win[4 * m + 1] = v.y; win[4 * m + 2] = v.z; win[4 * m + 3] = v.w;
            }
#pragma unroll
            for (int py = 0; py < PY; ++py) {
                const int j = q - py;
                if (j < 0 || j >= N) continue;
                const float* wj = w + j * N;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const float c = wj[i];
#pragma unroll
                    for (int px = 0; px < PX; ++px) acc[py][px] = fmaf(c, win[RA - R + px + i], acc[py][px]);
                }
            }
        }
    }

    const int xb = x0 + tx * PX;
#pragma unroll
    for (int py = 0; py < PY; ++py) {
        const int y = y0 + ty * PY + py;
        if (y >= H) break;
        const size_t row = (size_t)y * dp;
        if (vec_ok && xb + PX <= W && PX % 4 == 0) {
#pragma unroll
            for (int px = 0; px < PX; px += 4)
                store4<T>(dst, row + (size_t)(xb + px) * T::size,
                          mk4(acc[py][px], acc[py][px + 1], acc[py][px + 2], acc[py][px + 3]));
        } else {
#pragma unroll
            for (int px = 0; px < PX; ++px)
                if (xb + px < W) store_px<T>(dst, row + (size_t)(xb + px) * T::size, acc[py][px]);
        }
    }
}

template <class T, int R, int PX, int PY, int ORD>
hipError_t launch_lds_TR(const Conv2dArgs& a) {
    using G = Tile2d<R, PX, PY>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + G::TH - 1) / G::TH;
    const size_t al = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0) && ((uintptr_t)a.dst % al == 0) &&
                       (a.dp % al == 0);
    hipLaunchKernelGGL((conv2d_lds<T, R, PX, PY, ORD>), dim3(tiles_x * tiles_y), dim3(256), 0, a.st, a.src, a.sp,
                       a.dst, a.dp, a.W, a.H, a.taps, tiles_x, vec_ok, a.bd);
    return hipGetLastError();
}

template <class T, int PX, int PY, int ORD>
hipError_t launch_lds_T(const Conv2dArgs& a) {
    switch (a.r) {
        case 0: return launch_lds_TR<T, 0, PX, PY, ORD>(a);
        case 1: return launch_lds_TR<T, 1, PX, PY, ORD>(a);
        case 2: return launch_lds_TR<T, 2, PX, PY, ORD>(a);
        case 3: return launch_lds_TR<T, 3, PX, PY, ORD>(a);
        case 4: return launch_lds_TR<T, 4, PX, PY, ORD>(a);
        case 5: return launch_lds_TR<T, 5, PX, PY, ORD>(a);
        case 6: return launch_lds_TR<T, 6, PX, PY, ORD>(a);
        case 7: return launch_lds_TR<T, 7, PX, PY, ORD>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int PX, int PY, int ORD>
hipError_t launch_lds(const Conv2dArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_lds_T<F32, PX, PY, ORD>(a);
        case ICL_F16: return launch_lds_T<F16, PX, PY, ORD>(a);
        default: return launch_lds_T<BF16, PX, PY, ORD>(a);
    }
}

bool supports_lds(const Conv2dArgs& a) { return a.r >= 0 && a.r <= 7; }

// ------------------------------------------------------------------ persistent, prefetching, taps in LDS
// Each block walks tiles with stride gridDim.x.  While tile t is computed from LDS
// the global loads of tile t + gridDim.x are in flight in registers, so the HBM
// latency hides under the FMAs.  The taps live in LDS (read as broadcast float4)
// rather than SGPRs: a scalar load inside the loop forces a wait on every
// outstanding LDS read.  Tap rows are the outer loop; the PY input-row windows a
// lane needs form a rolling register buffer, so each staged row is read once.
template <class T, int R, int PX, int PY>
__global__ __launch_bounds__(256) void conv2d_pers(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                   size_t dp, int W, int H, const float* __restrict__ w, int tiles_x,
                                                   int tiles_y, int vec_ok, Border bd) {
    using G = Tile2d<R, PX, PY>;
    constexpr int TW = G::TW, TH = G::TH, RA = G::RA, LW = G::LW, NR = G::NR;
    constexpr int N = 2 * R + 1, NP = (N + 3) & ~3;
    __shared__ __attribute__((aligned(16))) float s[NR * LW];
    __shared__ __attribute__((aligned(16))) float wl[N * NP];
    const int tid = threadIdx.x;
    taps_to_lds<R, false>(w, 1, wl);
    Stage<T, NR, LW> st;
    const BandWalk walk(tiles_x, tiles_y);
    int t = walk.tile(0);
    if (t < 0) return;
    int x0, y0;
    tile_origin(t, tiles_x, TW, TH, x0, y0);
    st.load(src, sp, W, H, x0 - RA, y0 - R, vec_ok, bd);
    st.store(s);
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    for (int k = 0; t >= 0; ++k) {
        const int tn = walk.tile(k + 1);
        if (tn >= 0) {
            int nx0, ny0;
            tile_origin(tn, tiles_x, TW, TH, nx0, ny0);
            st.load(src, sp, W, H, nx0 - RA, ny0 - R, vec_ok, bd);
        }
        float acc[PY][PX];
#pragma unroll
        for (int py = 0; py < PY; ++py)
#pragma unroll
            for (int px = 0; px < PX; ++px) acc[py][px] = 0.f;
        corr_rows<R, PX, PY, LW>(&s[(ty * PY) * LW + tx * PX], wl, acc);
        __syncthreads();                 // every lane is done reading s
        if (tn >= 0) st.store(s);        // waits on the prefetch loads only: no output store issued yet
        const int xb = x0 + tx * PX;
#pragma unroll
        for (int py = 0; py < PY; ++py) {
            const int y = y0 + ty * PY + py;
            if (y >= H) break;
            const size_t row = (size_t)y * dp;
            if (vec_ok && xb + PX <= W) {
#pragma unroll
                for (int px = 0; px < PX; px += 4)
                    store4<T>(dst, row + (size_t)(xb + px) * T::size,
                              mk4(acc[py][px], acc[py][px + 1], acc[py][px + 2], acc[py][px + 3]));
            } else {
#pragma unroll
                for (int px = 0; px < PX; ++px)
                    if (xb + px < W) store_px<T>(dst, row + (size_t)(xb + px) * T::size, acc[py][px]);
            }
        }
        __syncthreads();                 // s holds the next tile
        t = tn;
        if (t >= 0) tile_origin(t, tiles_x, TW, TH, x0, y0);
    }
}

template <class T, int R, int PX, int PY>
hipError_t launch_pers_TR(const Conv2dArgs& a) {
    using G = Tile2d<R, PX, PY>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + G::TH - 1) / G::TH;
    const int ntiles = tiles_x * tiles_y;
    const size_t al = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0) && ((uintptr_t)a.dst % al == 0) &&
                       (a.dp % al == 0);
    const void* k = reinterpret_cast<const void*>(&conv2d_pers<T, R, PX, PY>);
    const int grid = persistent_grid(k, 256, ntiles);
    hipLaunchKernelGGL((conv2d_pers<T, R, PX, PY>), dim3(grid), dim3(256), 0, a.st, a.src, a.sp, a.dst, a.dp, a.W,
                       a.H, a.taps, tiles_x, tiles_y, vec_ok, a.bd);
    return hipGetLastError();
}

template <class T, int PX, int PY>
hipError_t launch_pers_T(const Conv2dArgs& a) {
    switch (a.r) {
        case 0: return launch_pers_TR<T, 0, PX, PY>(a);
        case 1: return launch_pers_TR<T, 1, PX, PY>(a);
        case 2: return launch_pers_TR<T, 2, PX, PY>(a);
        case 3: return launch_pers_TR<T, 3, PX, PY>(a);
        case 4: return launch_pers_TR<T, 4, PX, PY>(a);
        case 5: return launch_pers_TR<T, 5, PX, PY>(a);
        case 6: return launch_pers_TR<T, 6, PX, PY>(a);
        case 7: return launch_pers_TR<T, 7, PX, PY>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int PX, int PY>
hipError_t launch_pers(const Conv2dArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_pers_T<F32, PX, PY>(a);
        case ICL_F16: return launch_pers_T<F16, PX, PY>(a);
        default: return launch_pers_T<BF16, PX, PY>(a);
    }
}

const Variant<Conv2dArgs> kConv2d[] = {
    {"plain", supports_plain, launch_plain},
    {"lds_p4x4_o0", supports_lds, launch_lds<4, 4, 0>},
    {"lds_p4x4_o1", supports_lds, launch_lds<4, 4, 1>},
    {"lds_p4x8_o0", supports_lds, launch_lds<4, 8, 0>},
    {"lds_p4x2_o1", supports_lds, launch_lds<4, 2, 1>},
    {"lds_p8x2_o0", supports_lds, launch_lds<8, 2, 0>},
    {"pers_p4x4", supports_lds, launch_pers<4, 4>},
    {"pers_p8x2", supports_lds, launch_pers<8, 2>},
    {"pers_p4x2", supports_lds, launch_pers<4, 2>},
    {"pers_p8x4", supports_lds, launch_pers<8, 4>},
    {"mfma_f16x3", supports_conv2d_mfma, launch_conv2d_mfma},
};

}  // namespace

const Variant<Conv2dArgs>* conv2d_variants(int* count) {
    *count = (int)(sizeof(kConv2d) / sizeof(kConv2d[0]));
    return kConv2d;
}

int conv2d_default(const Conv2dArgs& a) { return supports_lds(a) ? 1 : 0; }

}  // namespace icl
