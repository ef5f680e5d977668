// Register-blocked correlation of an LDS tile with taps held in LDS, shared by the
// persistent 2-D and filter-bank kernels.
#pragma once
#include "icl_device.hpp"

namespace icl {

// Taps row j (N taps, zero-padded to NP) are read as broadcast float4 from LDS; the
// tap rows are the outer loop and the PY staged input rows a lane needs form a rolling
// register buffer, so each row window (PX + 2*RA floats, float4-aligned) is read once.
// `base` points at the lane's first window: staged row ty*PY, column tx*PX.
template <int R, int PX, int PY, int LW, bool SCHED_FENCE = false>
__device__ __forceinline__ void corr_rows(const float* __restrict__ base, const float* __restrict__ wl,
                                          float (&acc)[PY][PX]) {
    constexpr int N = 2 * R + 1, NP = (N + 3) & ~3, RA = (R + 3) & ~3, WIN = PX + 2 * RA;
    float win[PY][WIN];
    auto load_win = [&](float* dstw, const float* p) {
#pragma unroll
        for (int m = 0; m < WIN / 4; ++m) {
            const v4f v = lds4(p + 4 * m);
            dstw[4 * m] = v.x; dstw[4 * m + 1] = v.y; dstw[4 * m + 2] = v.z; dstw[4 * m + 3] = v.w;
        }
    };
#pragma unroll
    for (int py = 0; py < PY - 1; ++py) load_win(win[py], base + py * LW);
#pragma unroll 1
    for (int jb = 0; jb < N; jb += PY) {
#pragma unroll
        for (int u = 0; u < PY; ++u) {
            const int j = jb + u;
            if (j < N) {
                load_win(win[(u + PY - 1) % PY], base + (j + PY - 1) * LW);
                float tp[NP];
#pragma unroll
                for (int m = 0; m < NP / 4; ++m) {
                    const v4f v = lds4(&wl[j * NP + 4 * m]);
                    tp[4 * m] = v.x; tp[4 * m + 1] = v.y; tp[4 * m + 2] = v.z; tp[4 * m + 3] = v.w;
                }
#pragma unroll
                for (int py = 0; py < PY; ++py) {
                    const float* wv = win[(u + py) % PY];
#pragma unroll
                    for (int i = 0; i < N; ++i)
#pragma unroll
                        for (int px = 0; px < PX; ++px) acc[py][px] = fmaf(tp[i], wv[RA - R + px + i], acc[py][px]);
                }
                // keep the next row's LDS reads from being hoisted above these FMAs: hoisting
                // them all multiplies the live window registers and costs occupancy
                if constexpr (SCHED_FENCE) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// Copy F filters of N x N taps (row major, contiguous) into LDS rows padded to NP;
// FLIP stores each filter rotated by 180 degrees (the adjoint's flipped filter).
template <int R, bool FLIP>
__device__ __forceinline__ void taps_to_lds(const float* __restrict__ w, int F, float* __restrict__ wl) {
    constexpr int N = 2 * R + 1, NP = (N + 3) & ~3;
    for (int i = threadIdx.x; i < F * N * NP; i += blockDim.x) {
        const int f = i / (N * NP), rem = i - f * N * NP, j = rem / NP, c = rem - j * NP;
        float v = 0.f;
        if (c < N) v = FLIP ? w[f * N * N + (N - 1 - j) * N + (N - 1 - c)] : w[f * N * N + j * N + c];
        wl[i] = v;
    }
}

}  // namespace icl
