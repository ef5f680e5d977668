// Register-streaming separable correlation: one wave owns a strip of columns and walks
// down its rows.  Shared by the per-image and batched kernels.
//
// Lane l holds the four columns xs - RA + 4l .. xs - RA + 4l + 3 of every input row it
// walks (RA = r rounded up to whole lanes of four columns).  The HL = RA/4 lanes at each
// end of the wave only supply the horizontal halo; the others own SW = 4 (64 - 2 HL)
// output columns.  Columns outside the image are loaded clamped (or as the constant of a
// constant boundary), which is exactly the row pass's boundary, so the first and last
// strip of an image need no special path.
//
// Per input row (image row clamp(y0 - r + kk)):
//   * its four columns arrive from a ring of prefetched rows (Q rows ahead);
//   * the horizontal pass takes the neighbouring lanes' columns through DPP wave shifts
//     and sums taps_x in ascending order, fmaf from zero (the row pass's order);
//   * the row is added, weighted by taps_y[j], into the pending output row kk - j for
//     j = 0 .. 2r (a ring of 2r+1 float4 accumulators; the column pass's order);
//   * output row kk - 2r is then complete and is written.
// So every output is the same float32 expression as in the LDS tile kernels: the
// variants agree bit for bit.
#pragma once
#include "icl_device.hpp"

namespace icl {

template <int R> struct StripGeom {
    static constexpr int RA = (R + 3) & ~3;              // halo columns per side
    static constexpr int HL = RA / 4;                     // halo lanes per side
    static constexpr int SW = 4 * (64 - 2 * HL);          // output columns per strip
    static constexpr int D = 2 * R + 1;                   // pending output rows
    static constexpr int U = D * ((8 + D - 1) / D);       // unroll: constant ring slots
    static constexpr int Q = R <= 2 ? 8 : (R <= 4 ? 6 : 4);   // rows in flight ahead
    static_assert(Q <= U, "prefetch distance must fit the ring");
};

// Horizontal pass of one row: v holds this lane's four columns.
template <int R>
__device__ __forceinline__ v4f strip_row_pass(const v4f v, const float* __restrict__ tx) {
    using G = StripGeom<R>;
    constexpr int RA = G::RA;
    float e[4 + 2 * RA];
    e[RA] = v.x; e[RA + 1] = v.y; e[RA + 2] = v.z; e[RA + 3] = v.w;
    if constexpr (RA >= 4) {
        // lane - 1 and lane + 1 (only the columns within r of this lane's are used)
        float l1[4], r1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (RA - 4 + i >= RA - R) l1[i] = lane_from_left(v[i]);
            if (i < R) r1[i] = lane_from_right(v[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (RA - 4 + i >= RA - R) e[RA - 4 + i] = l1[i];
            if (i < R) e[RA + 4 + i] = r1[i];
        }
        if constexpr (RA >= 8) {
            // lane - 2 and lane + 2: shift the lane +-1 values once more
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (RA - 8 + i >= RA - R) e[RA - 8 + i] = lane_from_left(l1[i]);
                if (4 + i < R) e[RA + 8 + i] = lane_from_right(r1[i]);
            }
        }
    }
    float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) {
        const float h = tx[i];
#pragma unroll
        for (int p = 0; p < 4; ++p) o[p] = fmaf(h, e[RA - R + p + i], o[p]);
    }
    return mk4(o[0], o[1], o[2], o[3]);
}

// One strip: output columns xs .. xs + SW - 1 (those below W) and rows y0 .. y0 + TH - 1
// (those below H).  vec_in / vec_out: rows start 4-pixel aligned (16 B for float32).
template <class T, int R, int TH>
__device__ __forceinline__ void sep_strip_body(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                               size_t dp, int W, int H, const float* __restrict__ tx,
                                               const float* __restrict__ ty, int xs, int y0, bool vec_in,
                                               bool vec_out, Border bd = {}) {
    using G = StripGeom<R>;
    constexpr int D = G::D, U = G::U, Q = G::Q, HL = G::HL;
    constexpr int K = TH + 2 * R;   // input rows walked
    const int lane = threadIdx.x & 63;
    const int c = xs - G::RA + 4 * lane;
    const bool inside = vec_in && c >= 0 && c + 4 <= W;
    const int c0 = clampi(c, W), c1 = clampi(c + 1, W), c2 = clampi(c + 2, W), c3 = clampi(c + 3, W);
    // a column outside the image reads the constant (constant boundary) or its clamped pixel
    const bool o0 = bd.constant && (c < 0 || c >= W), o1 = bd.constant && (c + 1 < 0 || c + 1 >= W);
    const bool o2 = bd.constant && (c + 2 < 0 || c + 2 >= W), o3 = bd.constant && (c + 3 < 0 || c + 3 >= W);
    auto load_row = [&](int kk) -> v4f {
        const int yy = y0 - R + kk;
        if (bd.constant && (yy < 0 || yy >= H)) return mk4(bd.value, bd.value, bd.value, bd.value);
        const size_t row = (size_t)clampi(yy, H) * sp;
        if (inside) return load4<T>(src, row + (size_t)c * T::size);
        return mk4(o0 ? bd.value : load_px<T>(src, row + (size_t)c0 * T::size),
                   o1 ? bd.value : load_px<T>(src, row + (size_t)c1 * T::size),
                   o2 ? bd.value : load_px<T>(src, row + (size_t)c2 * T::size),
                   o3 ? bd.value : load_px<T>(src, row + (size_t)c3 * T::size));
    };
    const bool writer = lane >= HL && lane < 64 - HL && c < W;
    const bool wvec = vec_out && c + 4 <= W;
    v4f ring[U];
#pragma unroll
    for (int i = 0; i < Q; ++i) ring[i] = i < K ? load_row(i) : mk4(0.f, 0.f, 0.f, 0.f);
    v4f acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = mk4(0.f, 0.f, 0.f, 0.f);
    for (int kb = 0; kb < K; kb += U) {
        static_for<U>([&](auto u_c) {
            constexpr int u = decltype(u_c)::value;
            const int kk = kb + u;
            if (kk >= K) return;
            const v4f hrow = strip_row_pass<R>(ring[u], tx);
            if (kk + Q < K) ring[(u + Q) % U] = load_row(kk + Q);   // that slot's row is consumed
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int m = kk - j;
                if (m < 0 || m >= TH) continue;
                const float w = ty[j];
                v4f& a = acc[((u - j) % D + D) % D];
                a.x = fmaf(w, hrow.x, a.x);
                a.y = fmaf(w, hrow.y, a.y);
                a.z = fmaf(w, hrow.z, a.z);
                a.w = fmaf(w, hrow.w, a.w);
            }
            if (kk >= 2 * R) {
                constexpr int slot = ((u - 2 * R) % D + D) % D;
                const int y = y0 + kk - 2 * R;
                if (writer && y < H) {
                    const size_t row = (size_t)y * dp;
                    const v4f a = acc[slot];
                    if (wvec) {
                        store4<T>(dst, row + (size_t)c * T::size, a);
                    } else {
                        store_px<T>(dst, row + (size_t)c * T::size, a.x);
                        if (c + 1 < W) store_px<T>(dst, row + (size_t)(c + 1) * T::size, a.y);
                        if (c + 2 < W) store_px<T>(dst, row + (size_t)(c + 2) * T::size, a.z);
                        if (c + 3 < W) store_px<T>(dst, row + (size_t)(c + 3) * T::size, a.w);
                    }
                }
                acc[slot] = mk4(0.f, 0.f, 0.f, 0.f);
            }
        });
    }
}

}  // namespace icl
