// 2-D correlation on the matrix cores (radius 0..7).  Per tap row j the correlation of a
// 16 x 16 output block is a product with a banded (Toeplitz) tap matrix:
//   out[m][n] += sum_k X[m + j][k] * B_j[k][n],   B_j[k][n] = w[j][k - n] (0 <= k - n <= 2r)
// with k running over the 32 input columns that feed the block (16 + 2r <= 32).  The
// float32 operands are split into two float16 halves (x = hi + lo, hi = fp16(x),
// lo = fp16(x - hi)) and each product is hi*hi + hi*lo + lo*hi in v_mfma_f32_16x16x32_f16
// with float32 accumulation: the dropped lo*lo term and the two splitting roundings stay below
// 2^-20 of |x w|, far inside the float32 tolerance of the other variants.  So that float16
// range holds any finite input, the staged pixels of each tile and the taps are scaled by
// powers of two (exact) from their largest magnitudes and the sums unscaled.
//
// Lane layouts (checked with an in-bounds probe): A[i][k] lane i + 16 (k / 8), element k % 8;
// B[k][j] lane j + 16 (k / 8), element k % 8; D[i][j] lane j + 16 (i / 4), register i % 4.
//
// Persistent work-groups of 256 lanes walk 64 x 64 output tiles (column bands per XCD, so
// that halo rows are shared in one L2); wave w takes rows 16w .. 16w + 15 of a tile as four
// 16 x 16 blocks, and the next tile's pixels are loaded into registers while the products of
// the current one run.  The tap scale and tables are built once per work-group.  LDS: the staged tile as float16 hi and lo planes ((64 + 2r) rows x 80
// columns from the 4-aligned column x0 - RA, RA = r rounded up to a multiple of 4, rows
// padded to 88 halves so that the 16-byte reads of consecutive rows fall in distinct banks)
// and the Toeplitz tables of every tap row (hi and lo, lane order), which absorb the
// RA - r column offset.  Each wave reads the operands of tap row j + 1 while the products
// of row j run.
// Operand error (besides the float32 accumulation rounding all variants have): at most
// 2^-20 sum|x w| + 2^-37 (2r+1)^2 M max|w|, M the largest |x| of the staged tile.  The second
// term comes from float16's exponent range: a pixel (tap) more than about 2^20 below the
// tile's (filter's) largest keeps fewer bits.  It matters only where a whole window is that
// small next to a bright one (the FMA variants have no such term), so the variant is never
// the default: the tuner may pick it.  It assumes finite pixels and taps (a non-finite value
// spoils its whole tile).
#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "tile_stage.hpp"

namespace icl {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

constexpr int MT = 64;                  // output tile side
constexpr int LWH = 80;                 // staged columns: block cb reads 16 cb .. 16 cb + 31
constexpr int NC4 = LWH / 4;            // float4 chunks per staged row
constexpr int LWP = 88;                 // staged row pitch (halves): 176 B, an odd number of 16 B
template <int R> struct MTile {
    static constexpr int N = 2 * R + 1;
    static constexpr int NR = MT + 2 * R;               // staged rows
    static constexpr int RA = (R + 3) & ~3;             // staged column 0 is input column x0 - RA
    static constexpr int SH = RA - R;                    // staged columns before x0 - r
    static_assert(15 + SH + 2 * R < 32, "a block's taps must fit its 32 staged columns");
    static_assert(MT - 1 + RA + R < LWH, "the staged row must cover the right halo");
};

__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    return m;
}

// exponent e = 13 - floor(log2 m): m * 2^e lies in [2^13, 2^14).  Scaling goes through
// ldexpf, so an exponent beyond the float range (subnormal m) is still applied exactly.
__device__ __forceinline__ int pow2_exp(float m) { return m > 0.f ? 13 - ilogbf(m) : 0; }

// Up to r = 5 the LDS tile leaves room for three work-groups per CU, so the register budget is
// set for three waves per SIMD; wider windows keep two.
template <class T, int R>
__global__ __launch_bounds__(256, (R <= 5 ? 3 : 2)) void conv2d_mfma_k(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                     size_t dp, int W, int H, const float* __restrict__ taps,
                                                     int tiles_x, int tiles_y, int vec_in, Border bd) {
    using G = MTile<R>;
    constexpr int N = G::N, NR = G::NR, SH = G::SH, RA = G::RA;
    constexpr int NCH = NR * NC4, PER = (NCH + 255) / 256;
    __shared__ __attribute__((aligned(16))) _Float16 xh[NR * LWP];
    __shared__ __attribute__((aligned(16))) _Float16 xl[NR * LWP];
    __shared__ __attribute__((aligned(16))) h8 bh[N * 64];
    __shared__ __attribute__((aligned(16))) h8 bl[N * 64];
    __shared__ float wsh[N * N];
    __shared__ float red[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BandWalk walk(tiles_x, tiles_y);
    int t = walk.tile(0);
    if (t < 0) return;   // the whole work-group

    // taps, their scale, and the Toeplitz tables (once per work-group): entry (j, lane) holds
    // the eight taps w[j][8 (lane / 16) + e - lane % 16 - SH], e = 0..7 (zero outside 0..2r)
    float wm = 0.f;
    for (int k = tid; k < N * N; k += 256) {
        const float v = taps[k];
        wsh[k] = v;
        wm = fmaxf(wm, fabsf(v));
    }
    const int ew = pow2_exp(block_max(wm, red));   // also orders wsh before its reads
    for (int e = tid; e < N * 64; e += 256) {
        const int j = e / 64, l = e % 64;
        h8 hi, lo;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int tt = 8 * (l / 16) + q - (l % 16) - SH;
            const float v = (tt >= 0 && tt < N) ? ldexpf(wsh[j * N + tt], ew) : 0.f;
            const _Float16 h = (_Float16)v;
            hi[q] = h;
            lo[q] = (_Float16)(v - (float)h);
        }
        bh[e] = hi;
        bl[e] = lo;
    }

    // stage rows y0-r .. y0+63+r, columns x0-RA .. x0-RA+79 of a tile into registers through
    // the boundary condition.  A tile whose staged region lies inside the image (rows 16-byte
    // aligned) loads float4 chunks; the others load element by element.
    v4f v[PER];
    auto interior = [&](int x0, int y0) {
        return vec_in && x0 - RA >= 0 && x0 - RA + LWH <= W && y0 - R >= 0 && y0 - R + NR <= H;
    };
    auto load_tile = [&](int x0, int y0) {
        if (interior(x0, y0)) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int c = tid + 256 * i;
                if (c >= NCH) break;
                const int rr = c / NC4, c4 = c - rr * NC4;
                v[i] = load4<T>(src, (size_t)(y0 - R + rr) * sp + (size_t)(x0 - RA + 4 * c4) * T::size);
            }
            return;
        }
        // edge tile: every element from its clamped address, with no branches between the
        // loads so that they are all in flight together (a constant boundary is applied when
        // the tile is consumed)
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid + 256 * i;
            if (c >= NCH) break;
            const int rr = c / NC4, c4 = c - rr * NC4;
            const int yy = y0 - R + rr, xx = x0 - RA + 4 * c4;
            const size_t row = (size_t)clampi(yy, H) * sp;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[i][q] = load_px<T>(src, row + (size_t)clampi(xx + q, W) * T::size);
        }
    };
    int x0, y0;
    tile_origin(t, tiles_x, MT, MT, x0, y0);
    load_tile(x0, y0);

    const int m = lane & 15, kq = lane >> 4;
    for (int k = 0; t >= 0; ++k) {
        // scale of this tile; block_max's first barrier also orders the previous tile's
        // operand reads before the staging writes below
        if (bd.constant && !interior(x0, y0)) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int c = tid + 256 * i;
                if (c >= NCH) break;
                const int rr = c / NC4, c4 = c - rr * NC4;
                const int yy = y0 - R + rr, xx = x0 - RA + 4 * c4;
                const bool rowout = yy < 0 || yy >= H;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (rowout || xx + q < 0 || xx + q >= W) v[i][q] = bd.value;
            }
        }
        float xm = 0.f;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (tid + 256 * i >= NCH) break;
            xm = fmaxf(xm, fmaxf(fmaxf(fabsf(v[i].x), fabsf(v[i].y)), fmaxf(fabsf(v[i].z), fabsf(v[i].w))));
        }
        const int ex = pow2_exp(block_max(xm, red));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid + 256 * i;
            if (c >= NCH) break;
            const int rr = c / NC4, c4 = c - rr * NC4;
            h4 hi, lo;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float sv = ldexpf(v[i][q], ex);
                hi[q] = (_Float16)sv;
                lo[q] = (_Float16)(sv - (float)hi[q]);
            }
            *reinterpret_cast<h4*>(&xh[rr * LWP + 4 * c4]) = hi;
            *reinterpret_cast<h4*>(&xl[rr * LWP + 4 * c4]) = lo;
        }
        __syncthreads();
        // the next tile's loads run under this tile's products
        const int tn = walk.tile(k + 1);
        int nx0 = 0, ny0 = 0;
        if (tn >= 0) {
            tile_origin(tn, tiles_x, MT, MT, nx0, ny0);
            load_tile(nx0, ny0);
        }

        // products: block (wave, cb) covers output rows 16 wave + 0..15, columns 16 cb + 0..15;
        // the operands of tap row j + 1 are read into the other buffer before row j's products
        v4f acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = mk4(0.f, 0.f, 0.f, 0.f);
        h8 b_hi[2], b_lo[2], a_hi[2][4], a_lo[2][4];
        auto fetch = [&](int j, int buf) {
            b_hi[buf] = bh[j * 64 + lane];
            b_lo[buf] = bl[j * 64 + lane];
            const int arow = (16 * wave + m + j) * LWP + 8 * kq;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                a_hi[buf][cb] = *reinterpret_cast<const h8*>(&xh[arow + 16 * cb]);
                a_lo[buf][cb] = *reinterpret_cast<const h8*>(&xl[arow + 16 * cb]);
            }
        };
        fetch(0, 0);
        static_for<N>([&](auto j_c) {
            constexpr int j = decltype(j_c)::value, cur = j & 1;
            if constexpr (j + 1 < N) fetch(j + 1, cur ^ 1);
            __builtin_amdgcn_sched_barrier(0);   // keep the next row's reads ahead of these products
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_hi[cur][cb], b_hi[cur], acc[cb], 0, 0, 0);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_hi[cur][cb], b_lo[cur], acc[cb], 0, 0, 0);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_lo[cur][cb], b_hi[cur], acc[cb], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        });

        // lane holds out[16 wave + 4 kq + i][16 cb + m] in acc[cb][i]
        const int eo = -(ex + ew);   // undo both scalings (exact)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int x = x0 + 16 * cb + m;
            if (x >= W) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = y0 + 16 * wave + 4 * kq + i;
                if (y < H) store_px<T>(dst, (size_t)y * dp + (size_t)x * T::size, ldexpf(acc[cb][i], eo));
            }
        }
        t = tn;
        x0 = nx0;
        y0 = ny0;
    }
}

template <class T, int R>
hipError_t launch_TR(const Conv2dArgs& a) {
    const long long tx = (a.W + MT - 1) / MT, ty = (a.H + MT - 1) / MT;
    if (tx * ty > 0x7fffffffLL) return hipErrorInvalidValue;
    const int tiles_x = (int)tx, tiles_y = (int)ty;
    const size_t al = 4 * (size_t)T::size;
    const int vec_in = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0);
    const void* k = reinterpret_cast<const void*>(&conv2d_mfma_k<T, R>);
    const int grid = persistent_grid(k, 256, tiles_x * tiles_y);
    hipLaunchKernelGGL((conv2d_mfma_k<T, R>), dim3(grid), dim3(256), 0, a.st, a.src, a.sp, a.dst, a.dp, a.W, a.H,
                       a.taps, tiles_x, tiles_y, vec_in, a.bd);
    return hipGetLastError();
}

template <class T>
hipError_t launch_T(const Conv2dArgs& a) {
    switch (a.r) {
        case 0: return launch_TR<T, 0>(a);
        case 1: return launch_TR<T, 1>(a);
        case 2: return launch_TR<T, 2>(a);
        case 3: return launch_TR<T, 3>(a);
        case 4: return launch_TR<T, 4>(a);
        case 5: return launch_TR<T, 5>(a);
        case 6: return launch_TR<T, 6>(a);
        case 7: return launch_TR<T, 7>(a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool supports_conv2d_mfma(const Conv2dArgs& a) { return a.r >= 0 && a.r <= 7; }

hipError_t launch_conv2d_mfma(const Conv2dArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_T<F32>(a);
        case ICL_F16: return launch_T<F16>(a);
        default: return launch_T<BF16>(a);
    }
}

}  // namespace icl
