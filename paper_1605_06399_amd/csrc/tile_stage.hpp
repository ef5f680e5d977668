// Persistent tile machinery shared by the stencil kernels.
//
// A staged tile is NR rows x LW columns of float32 (LW a multiple of 4) whose
// top-left element is image pixel (gx0, gy0).  Stage<> loads it from global
// memory into registers (float4 per slot, 256 lanes), so the loads of the NEXT
// tile can be in flight while the current one is computed from LDS, and then
// writes the registers to LDS.  Reads outside the image follow the clamped
// boundary (or read zero with ZERO_PAD).
#pragma once
#include "icl_device.hpp"

namespace icl {

template <class T, int NR, int LW, bool ZERO_PAD = false>
struct Stage {
    static constexpr int C4 = LW / 4;
    static constexpr int N = (NR * C4 + 255) / 256;
    v4f v[N];

    // vec: every column of the tile is inside the image and rows start 4-pixel aligned
    __device__ __forceinline__ void load(const void* __restrict__ src, size_t sp, int W, int H, int gx0, int gy0,
                                         bool vec) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int idx = (int)threadIdx.x + 256 * k;
            if (N * 256 != NR * C4 && idx >= NR * C4) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int yy = gy0 + rr;
            const int x = gx0 + 4 * c4;
            if (ZERO_PAD && (yy < 0 || yy >= H)) {
                v[k] = mk4(0.f, 0.f, 0.f, 0.f);
                continue;
            }
            const size_t row = (size_t)clampi(yy, H) * sp;
            if (vec) {
                v[k] = load4<T>(src, row + (size_t)x * T::size);
            } else {
                float e[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int xx = x + q;
                    e[q] = (ZERO_PAD && (xx < 0 || xx >= W)) ? 0.f
                                                             : load_px<T>(src, row + (size_t)clampi(xx, W) * T::size);
                }
                v[k] = mk4(e[0], e[1], e[2], e[3]);
            }
        }
    }

    __device__ __forceinline__ void store(float* __restrict__ s) const {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int idx = (int)threadIdx.x + 256 * k;
            if (N * 256 != NR * C4 && idx >= NR * C4) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            lds4(&s[rr * LW + 4 * c4], v[k]);
        }
    }
};

// Tile t of a tiles_x-wide row-major tiling -> top-left output pixel.
__device__ __forceinline__ void tile_origin(int t, int tiles_x, int tw, int th, int& x0, int& y0) {
    const int ty = t / tiles_x;
    x0 = (t - ty * tiles_x) * tw;
    y0 = ty * th;
}

// First tile of this block in a persistent walk (stride gridDim.x).  With a grid that
// is a multiple of 8, consecutive tiles of each round go to one XCD, so tiles sharing
// halo rows meet in the same L2.
__device__ __forceinline__ int first_tile() { return (int)xcd_remap(blockIdx.x, gridDim.x); }

}  // namespace icl
