// Fused single-pass separable tile, shared by the per-image and batched kernels.
#pragma once
#include "icl_device.hpp"

namespace icl {

// ------------------------------------------------------------------ fused tile (also used by the batched kernel)
// Geometry of one fused tile for radius R.
template <int R, int TH, int CX> struct SepTile {
    static constexpr int TW = 64 * CX;           // output columns
    static constexpr int RA = (R + 3) & ~3;      // column halo rounded up to whole float4s
    static constexpr int LW = TW + 2 * RA;       // staged input row length (floats)
    static constexpr int NR = TH + 2 * R;        // staged input rows
    static constexpr int LDS_FLOATS = NR * LW + NR * TW;
};

// Row pass over a staged tile: in_s [NR][LW] -> t_s [NR][TW], four columns per item.
// UNR > 0 caps the unrolling of the item loop (a trip count known at compile time is
// otherwise unrolled whole, with every item's window in registers at once).
template <int R, int TH, int CX, int UNR = 0>
__device__ __forceinline__ void sep_row_pass(const float* __restrict__ in_s, float* __restrict__ t_s,
                                             const float* __restrict__ tx) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR, G4 = TW / 4;
    auto item = [&](int idx) {
        const int rr = idx / G4, g = idx - rr * G4;
        float win[4 + 2 * RA];
#pragma unroll
        for (int m = 0; m < (4 + 2 * RA) / 4; ++m) {
            const v4f v = lds4(&in_s[rr * LW + 4 * g + 4 * m]);
            win[4 * m] = v.x; win[4 * m + 1] = v.y; win[4 * m + 2] = v.z; win[4 * m + 3] = v.w;
        }
        float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) {
            const float h = tx[i];
#pragma unroll
            for (int p = 0; p < 4; ++p) o[p] = fmaf(h, win[RA - R + p + i], o[p]);
        }
        lds4(&t_s[rr * TW + 4 * g], mk4(o[0], o[1], o[2], o[3]));
    };
    if constexpr (UNR > 0) {
#pragma unroll UNR
        for (int idx = threadIdx.x; idx < NR * G4; idx += 256) item(idx);
    } else {
        for (int idx = threadIdx.x; idx < NR * G4; idx += 256) item(idx);
    }
}

// Column pass: lane owns 4 adjacent columns (group g of TW/4) and PYC consecutive rows;
// the t_s rows it needs are read as float4, and the 4 outputs of a row are stored as one
// vector when the destination rows are 4-pixel aligned (vec_out).
// GROUP > 0 fences the schedule every GROUP staged rows, so that at most GROUP rows' reads are
// in registers at a time (a kernel that must fit a register budget).
template <class T, int R, int TH, int CX, int GROUP = 0>
__device__ __forceinline__ void sep_col_pass(const float* __restrict__ t_s, void* __restrict__ dst, size_t dp, int W,
                                             int H, const float* __restrict__ ty, int x0, int y0, bool vec_out) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, G4 = TW / 4, RPI = 256 / G4, PYC = TH / RPI;
    static_assert(PYC * RPI == TH, "tile rows must split evenly over the row groups");
    const int g = threadIdx.x % G4, rg = threadIdx.x / G4;
    const float* col = t_s + (rg * PYC) * TW + 4 * g;
    // each staged row is read once and added into every output row it feeds
    v4f acc[PYC];
#pragma unroll
    for (int py = 0; py < PYC; ++py) acc[py] = mk4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int m = 0; m < PYC + 2 * R; ++m) {
        if (GROUP > 0 && m > 0 && m % GROUP == 0) __builtin_amdgcn_sched_barrier(0);
        const v4f v = lds4(col + m * TW);
#pragma unroll
        for (int py = 0; py < PYC; ++py) {
            const int j = m - py;
            if (j < 0 || j > 2 * R) continue;
            const float c = ty[j];
            acc[py].x = fmaf(c, v.x, acc[py].x);
            acc[py].y = fmaf(c, v.y, acc[py].y);
            acc[py].z = fmaf(c, v.z, acc[py].z);
            acc[py].w = fmaf(c, v.w, acc[py].w);
        }
    }
    const int x = x0 + 4 * g;
#pragma unroll
    for (int py = 0; py < PYC; ++py) {
        const int y = y0 + rg * PYC + py;
        if (y >= H) break;
        const size_t row = (size_t)y * dp;
        const v4f a = acc[py];
        if (vec_out && x + 4 <= W) {
            store4<T>(dst, row + (size_t)x * T::size, a);
        } else {
            if (x < W) store_px<T>(dst, row + (size_t)x * T::size, a.x);
            if (x + 1 < W) store_px<T>(dst, row + (size_t)(x + 1) * T::size, a.y);
            if (x + 2 < W) store_px<T>(dst, row + (size_t)(x + 2) * T::size, a.z);
            if (x + 3 < W) store_px<T>(dst, row + (size_t)(x + 3) * T::size, a.w);
        }
    }
}

// Computes one TW x TH output tile whose top-left output pixel is (x0, y0), staging
// directly (no prefetch).  `lds` holds SepTile::LDS_FLOATS floats.  vec: interior-in-x
// tile with 4-pixel aligned rows, loaded with vector loads and no column clamps.
template <class T, int R, int TH, int CX>
__device__ __forceinline__ void sep_tile_body(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                              size_t dp, int W, int H, const float* __restrict__ tx,
                                              const float* __restrict__ ty, int x0, int y0, bool vec, bool vec_out,
                                              float* __restrict__ lds, Border bd = {}) {
    using G = SepTile<R, TH, CX>;
    constexpr int RA = G::RA, LW = G::LW, NR = G::NR;
    float* in_s = lds;             // [NR][LW]
    float* t_s = lds + NR * LW;    // [NR][TW]
    const int tid = threadIdx.x;
    if (vec) {   // the tile's columns are inside the image: only rows can be outside
        // every chunk's load is issued before any is written to LDS (a load-then-write loop
        // would wait on each load in turn); rows outside the image load their clamped row and
        // take the constant afterwards, so no branch separates the loads
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
    sep_row_pass<R, TH, CX>(in_s, t_s, tx);
    __syncthreads();
    sep_col_pass<T, R, TH, CX>(t_s, dst, dp, W, H, ty, x0, y0, vec_out);
}

}  // namespace icl
