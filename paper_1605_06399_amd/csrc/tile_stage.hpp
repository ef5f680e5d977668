// Persistent tile machinery shared by the stencil kernels.
//
// A staged tile is NR rows x LW columns of float32 (LW a multiple of 4) whose
// top-left element is image pixel (gx0, gy0).  Stage<> loads it from global
// memory into registers (float4 per slot, 256 lanes), so the loads of the NEXT
// tile can be in flight while the current one is computed from LDS, and then
// writes the registers to LDS.  Reads outside the image follow the boundary: clamp or a
// constant (Border), or zero with ZERO_PAD.
#pragma once
#include <type_traits>

#include "icl_device.hpp"

namespace icl {

template <class T, int NR, int LW, bool ZERO_PAD = false>
struct Stage {
    static constexpr int C4 = LW / 4;
    static constexpr int N = (NR * C4 + 255) / 256;
    v4f v[N];

    // One float4 chunk of staged row data starting at pixel x of a row.  With `aligned`
    // rows (4-pixel aligned base and pitch, x a multiple of 4) a chunk is either fully
    // inside the row (one vector load), fully outside (zeros, or the clamped edge pixel
    // broadcast), or straddles the right edge (per element; only when W % 4 != 0).
    // bd: the boundary of the convolution kernels (clamp or a constant); ZERO_PAD, the
    // adjoint's zero extension, takes precedence.
    __device__ __forceinline__ static v4f chunk(const void* __restrict__ src, size_t row, int W, int x, bool aligned,
                                                Border bd = {}) {
        if (aligned && x >= 0 && x + 4 <= W) return load4<T>(src, row + (size_t)x * T::size);
        if (aligned && (x + 4 <= 0 || x >= W)) {
            if (ZERO_PAD) return mk4(0.f, 0.f, 0.f, 0.f);
            if (bd.constant) return mk4(bd.value, bd.value, bd.value, bd.value);
            const float e = load_px<T>(src, row + (size_t)clampi(x, W) * T::size);
            return mk4(e, e, e, e);
        }
        float e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int xx = x + q;
            const bool out = xx < 0 || xx >= W;
            e[q] = (ZERO_PAD && out) ? 0.f
                   : (bd.constant && out) ? bd.value
                                          : load_px<T>(src, row + (size_t)clampi(xx, W) * T::size);
        }
        return mk4(e[0], e[1], e[2], e[3]);
    }

    // Load the tile with top-left pixel (gx0, gy0); gx0 must be a multiple of 4 when
    // `aligned` (rows 4-pixel aligned in memory).
    __device__ __forceinline__ void load(const void* __restrict__ src, size_t sp, int W, int H, int gx0, int gy0,
                                         bool aligned, Border bd = {}) {
        // A tile that lies inside the image (the work-group's usual case) takes straight vector
        // loads: no branch between them, so they are all in flight together.  The general path
        // below branches per chunk, and the compiler then waits on each chunk's loads.
        if (aligned && gx0 >= 0 && gx0 + LW <= W && gy0 >= 0 && gy0 + NR <= H) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int idx = (int)threadIdx.x + 256 * k;
                if (N * 256 != NR * C4 && idx >= NR * C4) break;
                const int rr = idx / C4, c4 = idx - rr * C4;
                v[k] = load4<T>(src, (size_t)(gy0 + rr) * sp + (size_t)(gx0 + 4 * c4) * T::size);
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int idx = (int)threadIdx.x + 256 * k;
            if (N * 256 != NR * C4 && idx >= NR * C4) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int yy = gy0 + rr;
            if (ZERO_PAD && (yy < 0 || yy >= H)) {
                v[k] = mk4(0.f, 0.f, 0.f, 0.f);
                continue;
            }
            if (bd.constant && (yy < 0 || yy >= H)) {
                v[k] = mk4(bd.value, bd.value, bd.value, bd.value);
                continue;
            }
            v[k] = chunk(src, (size_t)clampi(yy, H) * sp, W, gx0 + 4 * c4, aligned, bd);
        }
    }

    // Every element the constant c (a whole staged region outside the image).
    __device__ __forceinline__ void fill(float c) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = mk4(c, c, c, c);
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

// Persistent schedule over a tiles_x x tiles_y grid (tiles numbered row-major) that keeps
// halo reuse inside one L2: the grid is cut into 8 column bands, one per XCD (gfx950
// places work-group b on XCD b % 8), and the blocks of an XCD walk their band row by
// row.  A tile's upper neighbour was therefore processed on the same XCD shortly before,
// and the halo rows they share are served from that XCD's L2 rather than HBM.
struct BandWalk {
    int tiles_x, bx0, bw, nband, slot, nslots;
    __device__ __forceinline__ BandWalk(int tx, int ty) : tiles_x(tx) {
        const int g = (int)gridDim.x;
        // one band per XCD; fewer when the grid or the tile row is too small, so every
        // band owns at least one block and one column (every tile is covered exactly once)
        int nb = g < 8 ? g : 8;
        nb = nb < tx ? nb : tx;
        const int x = (int)blockIdx.x % nb;
        slot = (int)blockIdx.x / nb;
        nslots = g / nb + (x < g % nb ? 1 : 0);
        bx0 = x * tx / nb;
        bw = (x + 1) * tx / nb - bx0;
        nband = bw * ty;
    }
    // k-th tile of this block, or -1 when its band is exhausted
    __device__ __forceinline__ int tile(int k) const {
        const int j = k * nslots + slot;
        if (j >= nband) return -1;
        const int row = j / bw;
        return row * tiles_x + bx0 + (j - row * bw);
    }
};

}  // namespace icl

namespace icl {

// Staged tile whose shape is known only at run time (NR <= NRMAX rows, LW = 4*C4 <= 128
// columns), as in a batch whose images have different radii.  The 256 lanes form 8 rows
// x 32 float4 columns, so no division by the runtime row length is needed.
template <class T, int NRMAX>
struct RStage {
    static constexpr int K = (NRMAX + 7) / 8;
    static constexpr bool BF = std::is_same<T, BF16>::value;
    v4f v[K];
    bool raw = false;   // bfloat16 fast path: v[k].x, .y hold the four packed values, unpacked at store

    // vec: rows 4-pixel aligned in memory (gx0 a multiple of 4)
    __device__ __forceinline__ void load(const void* __restrict__ src, size_t sp, int W, int H, int gx0, int gy0,
                                         int NR, int C4, bool vec) {
        const int c4 = threadIdx.x & 31, ry = threadIdx.x >> 5;
        if (c4 >= C4) return;
        const int x = gx0 + 4 * c4;
        raw = false;
        // inside the image: straight vector loads, all in flight together (bfloat16 stays
        // packed until the LDS store, which keeps the registers of the walk in check)
        if (vec && gx0 >= 0 && gx0 + 4 * C4 <= W && gy0 >= 0 && gy0 + NR <= H) {
            raw = BF;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int rr = ry + 8 * k;
                if (rr >= NR) break;
                const size_t off = (size_t)(gy0 + rr) * sp + (size_t)x * T::size;
                if constexpr (BF) {
                    const v2u u = *reinterpret_cast<const v2u*>(static_cast<const char*>(src) + off);
                    v[k].x = __uint_as_float(u.x);
                    v[k].y = __uint_as_float(u.y);
                } else {
                    v[k] = load4<T>(src, off);
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int rr = ry + 8 * k;
            if (rr >= NR) break;
            v[k] = Stage<T, 1, 4>::chunk(src, (size_t)clampi(gy0 + rr, H) * sp, W, x, vec);
        }
    }

    __device__ __forceinline__ void store(float* __restrict__ s, int NR, int C4) const {
        const int c4 = threadIdx.x & 31, ry = threadIdx.x >> 5;
        if (c4 >= C4) return;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int rr = ry + 8 * k;
            if (rr >= NR) break;
            v4f e = v[k];
            if (BF && raw) {
                const unsigned a = __float_as_uint(v[k].x), b = __float_as_uint(v[k].y);
                e = mk4(__uint_as_float(a << 16), __uint_as_float(a & 0xffff0000u), __uint_as_float(b << 16),
                        __uint_as_float(b & 0xffff0000u));
            }
            lds4(&s[rr * 4 * C4 + 4 * c4], e);
        }
    }
};

}  // namespace icl
