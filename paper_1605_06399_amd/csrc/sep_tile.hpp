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
    static constexpr int PY = TH / 4;            // column-pass rows per lane
    static constexpr int LDS_FLOATS = NR * LW + NR * TW;
};

// Row pass over a staged tile: in_s [NR][LW] -> t_s [NR][TW], four columns per item.
template <int R, int TH, int CX>
__device__ __forceinline__ void sep_row_pass(const float* __restrict__ in_s, float* __restrict__ t_s,
                                             const float* __restrict__ tx) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR, G4 = TW / 4;
    for (int idx = threadIdx.x; idx < NR * G4; idx += 256) {
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
    }
}

// Column pass: lane owns columns lx + 64c, rows ly*PY .. ly*PY+PY-1 of the tile at (x0, y0).
template <class T, int R, int TH, int CX>
__device__ __forceinline__ void sep_col_pass(const float* __restrict__ t_s, void* __restrict__ dst, size_t dp, int W,
                                             int H, const float* __restrict__ ty, int x0, int y0) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, PY = G::PY;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CX; ++c) {
        const int col = lx + 64 * c;
        float v[PY + 2 * R];
#pragma unroll
        for (int m = 0; m < PY + 2 * R; ++m) v[m] = t_s[(ly * PY + m) * TW + col];
        const int x = x0 + col;
#pragma unroll
        for (int py = 0; py < PY; ++py) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j <= 2 * R; ++j) acc = fmaf(ty[j], v[py + j], acc);
            const int y = y0 + ly * PY + py;
            if (x < W && y < H) store_px<T>(dst, (size_t)y * dp + (size_t)x * T::size, acc);
        }
    }
}

// Computes one TW x TH output tile whose top-left output pixel is (x0, y0), staging
// directly (no prefetch).  `lds` holds SepTile::LDS_FLOATS floats.  vec: interior-in-x
// tile with 4-pixel aligned rows, loaded with vector loads and no column clamps.
template <class T, int R, int TH, int CX>
__device__ __forceinline__ void sep_tile_body(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                              size_t dp, int W, int H, const float* __restrict__ tx,
                                              const float* __restrict__ ty, int x0, int y0, bool vec,
                                              float* __restrict__ lds) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR;
    float* in_s = lds;             // [NR][LW]
    float* t_s = lds + NR * LW;    // [NR][TW]
    const int tid = threadIdx.x;
    if (vec) {
        constexpr int C4 = LW / 4;
        for (int idx = tid; idx < NR * C4; idx += 256) {
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int y = clampi(y0 - R + rr, H);
            lds4(&in_s[rr * LW + 4 * c4], load4<T>(src, (size_t)y * sp + (size_t)(x0 - RA + 4 * c4) * T::size));
        }
    } else {
        for (int idx = tid; idx < NR * LW; idx += 256) {
            const int rr = idx / LW, c = idx - rr * LW;
            const int y = clampi(y0 - R + rr, H);
            const int x = clampi(x0 - RA + c, W);
            in_s[rr * LW + c] = load_px<T>(src, (size_t)y * sp + (size_t)x * T::size);
        }
    }
    __syncthreads();
    sep_row_pass<R, TH, CX>(in_s, t_s, tx);
    __syncthreads();
    sep_col_pass<T, R, TH, CX>(t_s, dst, dp, W, H, ty, x0, y0);
}

}  // namespace icl
