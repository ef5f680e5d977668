// Column walk of the separable filter, shared by the batched and the per-image kernels.
// A work-group walks one item: a strip of 64 CX columns of one image over a segment of rows,
// in steps of STEP output rows.  A step stages only the STEP input rows it adds, row-passes
// them into the T rows below the 2r T rows the previous step left (moved to the top), and
// column-passes STEP + 2r T rows.  So inside a segment every input row is loaded and
// row-passed once; a walk of separate tiles loads and row-passes STEP + 2r rows per STEP
// output rows.  Wider strips (CX = 2) halve the share of halo columns a strip reads.  The item body is instantiated per radius, with the same row and column
// passes, in the same tap order, as every other separable kernel, and either boundary.  The
// source is read through a buffer descriptor with 32-bit offsets.
#pragma once
#include "icl_device.hpp"
#include "sep_tile.hpp"

namespace icl {

// An image of a column walk (one image of a batch, or the single image of a call).
struct DevImage {
    const void* src;
    void* dst;
    unsigned long long sp, dp;
    const float* tx;
    const float* ty;
    int W, H, r, vec_ok, vec_out;
    unsigned src_bytes;   // extent of the source rows in bytes (the column walk's buffer size; 0 if >= 2^31)
};

// A column-walk item: output columns x0 .. x0 + 63 of image img over rows y0 .. y0 + rows - 1.
struct ColItem {
    int img, x0, y0, rows;
};


constexpr int COL_RMAX = 7;

// LDS of a column walk with strips of 64 CX columns and steps of STEP rows: the staged input
// rows of a step, the T rows of a step and its halo.
template <int CX, int STEP> struct ColGeom {
    static constexpr int CW = 64 * CX;
    static constexpr int LW_MAX = CW + 16;                    // staged row length at RA = 8 (floats)
    static constexpr int IN_FLOATS = STEP * LW_MAX;
    static constexpr int T_FLOATS = (STEP + 2 * COL_RMAX) * CW;
};

template <class T, int R, int NROWS, int CX = 1>
struct ColStage {
    static constexpr int RA = (R + 3) & ~3, LW = 64 * CX + 2 * RA, C4 = LW / 4;
    static constexpr int NCH = NROWS * C4, PER = (NCH + 255) / 256;
    typename Raw4<T>::type v[PER > 0 ? PER : 1];
    int gy = 0;

    // Staged rows gy .. gy + NROWS - 1 (read clamped into the image), columns x0 - RA .. x0 + 64 CX - 1 + RA.
    // inside (the columns lie in the image, rows 4-pixel aligned): straight vector loads into
    // registers, all in flight together, written to LDS by store().  Otherwise nothing is
    // loaded here: store() reads the chunks through the clamp itself (a strip at an image's
    // left or right edge, one in about eight), which keeps the rare edge path out of the
    // register budget of the prefetch.
    __device__ __forceinline__ void load(const DevImage& d, Rsrc rs, int x0, int row0, bool inside) {
        gy = row0;
        if (!inside) return;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int idx = (int)threadIdx.x + 256 * k;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            const unsigned row = (unsigned)clampi(gy + rr, d.H) * (unsigned)d.sp;
            v[k] = bload4_raw<T>(rs, row + (unsigned)(x0 - RA + 4 * c4) * T::size);
        }
    }
    // bd: the boundary; with a constant, a staged pixel outside the image is the constant
    __device__ __forceinline__ void store(float* __restrict__ in_s, const DevImage& d, Rsrc rs, int x0, bool inside,
                                          Border bd) const {
        if (inside) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int idx = (int)threadIdx.x + 256 * k;
                if (NCH % 256 != 0 && idx >= NCH) break;
                const int rr = idx / C4, c4 = idx - rr * C4;
                v4f e = decode4<T>(v[k]);
                if (bd.constant && (gy + rr < 0 || gy + rr >= d.H)) e = mk4(bd.value, bd.value, bd.value, bd.value);
                lds4(&in_s[rr * LW + 4 * c4], e);
            }
            return;
        }
        for (int idx = (int)threadIdx.x; idx < NCH; idx += 256) {
            const int rr = idx / C4, c4 = idx - rr * C4;
            const unsigned row = (unsigned)clampi(gy + rr, d.H) * (unsigned)d.sp;
            const int x = x0 - RA + 4 * c4;
            typename Raw4<T>::type r;
            if (d.vec_ok && x >= 0 && x + 4 <= d.W) {
                r = bload4_raw<T>(rs, row + (unsigned)x * T::size);
            } else {
                unsigned e[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) e[q] = bload1_raw<T>(rs, row + (unsigned)clampi(x + q, d.W) * T::size);
                r = pack4_raw<T>(e[0], e[1], e[2], e[3]);
            }
            v4f e = decode4<T>(r);
            if (bd.constant) {
                const bool yout = gy + rr < 0 || gy + rr >= d.H;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (yout || x + q < 0 || x + q >= d.W) e[q] = bd.value;
            }
            lds4(&in_s[rr * LW + 4 * c4], e);
        }
    }
};

// A value every lane loaded from the same address, moved to a scalar register: the item
// table and the images' descriptors and taps are read with vector loads (the compiler cannot
// prove that the kernel's stores leave them unchanged), and this keeps them out of the
// vector register budget.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
template <class P> __device__ __forceinline__ P* uni(P* p) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned long long lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned long long hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    return reinterpret_cast<P*>(lo | (hi << 32));
}
__device__ __forceinline__ DevImage uni(const DevImage& d) {
    DevImage u;
    u.src = uni(d.src); u.dst = uni(d.dst);
    u.sp = (unsigned long long)uni((int)d.sp) & 0xffffffffull;
    u.dp = ((unsigned long long)(unsigned)uni((int)(d.dp >> 32)) << 32) | (unsigned)uni((int)d.dp);
    u.tx = uni(d.tx); u.ty = uni(d.ty);
    u.W = uni(d.W); u.H = uni(d.H); u.r = uni(d.r); u.vec_ok = uni(d.vec_ok); u.vec_out = uni(d.vec_out);
    u.src_bytes = (unsigned)uni((int)d.src_bytes);
    return u;
}

template <class T, int R, int CX = 1, int STEP = 64>
__device__ __forceinline__ void col_item(const DevImage& d, const ColItem& it, float* __restrict__ in_s,
                                         float* __restrict__ t_s, Border bd = {}) {
    constexpr int RA = (R + 3) & ~3, CW = 64 * CX;
    const Rsrc rs = make_rsrc(d.src, d.src_bytes);
    float tx[2 * R + 1], ty[2 * R + 1];
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) {
        tx[i] = uni(d.tx[i]);
        ty[i] = uni(d.ty[i]);
    }
    const bool inside = d.vec_ok && it.x0 - RA >= 0 && it.x0 + CW + RA <= d.W;
    const int nsteps = (it.rows + STEP - 1) / STEP;
    // prologue: T rows 0 .. 2r - 1 from input rows y0 - r .. y0 + r - 1
    ColStage<T, R, STEP, CX> st;
    if constexpr (R > 0) {
        ColStage<T, R, 2 * R, CX> pro;
        pro.load(d, rs, it.x0, it.y0 - R, inside);
        st.load(d, rs, it.x0, it.y0 + R, inside);
        pro.store(in_s, d, rs, it.x0, inside, bd);
        __syncthreads();
        sep_row_pass<R, 0, CX, 1>(in_s, t_s, tx);
        __syncthreads();
    } else {
        st.load(d, rs, it.x0, it.y0 + R, inside);
    }
    for (int s = 0; s < nsteps; ++s) {
        st.store(in_s, d, rs, it.x0, inside, bd);
        if (R > 0 && s > 0) {   // the previous step's last 2r T rows become the first
            for (int q = (int)threadIdx.x; q < 2 * R * CW / 4; q += 256) lds4(&t_s[4 * q], lds4(&t_s[STEP * CW + 4 * q]));
        }
        __syncthreads();
        if (s + 1 < nsteps) st.load(d, rs, it.x0, it.y0 + STEP * (s + 1) + R, inside);
        sep_row_pass<R, STEP - 2 * R, CX, 1>(in_s, t_s + 2 * R * CW, tx);
        __syncthreads();
        sep_col_pass<T, R, STEP, CX, 6>(t_s, d.dst, d.dp, d.W, d.H, ty, it.x0, it.y0 + STEP * s, d.vec_out);
        __syncthreads();
    }
}

}  // namespace icl
