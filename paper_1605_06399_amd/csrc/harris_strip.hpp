// Register-strip building blocks shared by the Harris, NMS and fused corner kernels.
// A strip wave holds four adjacent columns per lane; neighbouring columns come from the
// adjacent lanes through DPP wave shifts.
#pragma once
#include "icl_device.hpp"

namespace icl {

// R = Sxx Syy - Sxy^2 - k (Sxx + Syy)^2 (Section 6, Harris corner detection)
__device__ __forceinline__ float harris_response(float sxx, float syy, float sxy, float k) {
    const float tr = sxx + syy;
    return sxx * syy - sxy * sxy - k * tr * tr;
}

// Horizontal window of radius RG over a lane's four columns, neighbours by DPP.
template <int RG>
__device__ __forceinline__ v4f hwin(v4f p, const float (&gw)[2 * RG + 1]) {
    float e[4 + 2 * RG];
#pragma unroll
    for (int i = 0; i < RG; ++i) e[i] = lane_from_left(p[4 - RG + i]);
    e[RG] = p.x; e[RG + 1] = p.y; e[RG + 2] = p.z; e[RG + 3] = p.w;
#pragma unroll
    for (int i = 0; i < RG; ++i) e[RG + 4 + i] = lane_from_right(p[i]);
    float o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t <= 2 * RG; ++t) acc = fmaf(gw[t], e[q + t], acc);
        o[q] = acc;
    }
    return mk4(o[0], o[1], o[2], o[3]);
}

// Gradient products of one row: Sobel from image rows ra (above), rb, rc (below), the
// neighbouring columns by DPP lane shifts; pa = Ix^2, pb = Iy^2, pc = Ix Iy.
__device__ __forceinline__ void sobel_products(const v4f ra, const v4f rb, const v4f rc, v4f& pa, v4f& pb, v4f& pc) {
    const v4f vs = ra + 2.f * rb + rc;   // vertical smoothing (for Ix)
    const v4f vd = rc - ra;              // vertical difference (for Iy)
    const float vsl = lane_from_left(vs.w), vsr = lane_from_right(vs.x);
    const float vdl = lane_from_left(vd.w), vdr = lane_from_right(vd.x);
    const v4f ix = mk4(vs.y - vsl, vs.z - vs.x, vs.w - vs.y, vsr - vs.z);
    const v4f iy = mk4(vdl + 2.f * vd.x + vd.y, vd.x + 2.f * vd.y + vd.z, vd.y + 2.f * vd.z + vd.w,
                       vd.z + 2.f * vd.w + vdr);
    pa = ix * ix;
    pb = iy * iy;
    pc = ix * iy;
}

// Products of one window row, then the horizontal window of each product.
template <int RG>
__device__ __forceinline__ void window_row(const v4f ra, const v4f rb, const v4f rc, const float (&gw)[2 * RG + 1],
                                           v4f& qa, v4f& qb, v4f& qc) {
    v4f pa, pb, pc;
    sobel_products(ra, rb, rc, pa, pb, pc);
    qa = hwin<RG>(pa, gw);
    qb = hwin<RG>(pb, gw);
    qc = hwin<RG>(pc, gw);
}

// NMS decision bits of a lane's four pixels of row b (rows a above, c below), radius 1:
// byte p of the result is 1 iff b[p] > tau and b[p] >= each of its eight neighbours.
__device__ __forceinline__ uint32_t nms_bits(v4f a, v4f b, v4f c, float tau) {
    const float al = lane_from_left(a.w), ar = lane_from_right(a.x);
    const float bl = lane_from_left(b.w), br = lane_from_right(b.x);
    const float cl = lane_from_left(c.w), cr = lane_from_right(c.x);
    const float ea[6] = {al, a.x, a.y, a.z, a.w, ar};
    const float eb[6] = {bl, b.x, b.y, b.z, b.w, br};
    const float ec[6] = {cl, c.x, c.y, c.z, c.w, cr};
    uint32_t bits = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float v = eb[p + 1];
        // bitwise & (no short circuit): nine compares, no branches
        const bool keep = (v > tau) & (v >= ea[p]) & (v >= ea[p + 1]) & (v >= ea[p + 2]) & (v >= eb[p]) &
                          (v >= eb[p + 2]) & (v >= ec[p]) & (v >= ec[p + 1]) & (v >= ec[p + 2]);
        bits |= (keep ? 1u : 0u) << (8 * p);
    }
    return bits;
}

}  // namespace icl
