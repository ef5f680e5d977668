// Fused corner detection: Harris response and 3x3 non-maximum suppression in one pass
// (Section 6 runs Harris as a Sobel kernel and a Harris kernel; its discussion names the
// fusion of such stages as the optimisation the language could not express).
//
//   mask(x,y) = 1 iff R(x,y) > tau and R(x,y) >= R at each of the 8 neighbours (reads of R
//               clamped to the image), with R the Harris response of icl_harris.
//
// The response never reaches HBM: 4 B/px in (image), 1 B/px out (mask), plus 4 B/px only
// when the caller asks for the response too.
//
// Variants
//   two_kernel : icl_harris then icl_nms through an intermediate response image (the caller's
//                response buffer or the workspace); any NMS radius.
//   stream_t{TH}: one wave per strip of 240 mask columns and TH rows (NMS radius 1, window
//                radius <= 3).  Lane l holds the image columns xm-8+4l .. xm-5+4l; lanes 1..62
//                form the response (their Harris window needs lanes 0..63), lanes 2..61 own
//                the mask (their NMS needs the response of lanes 1..62).  The wave walks the
//                window rows of the TH + 2 response rows y0-1 .. y0+TH; each finished
//                response row enters a ring of three, and the mask row above it is decided.
//                Strips and row blocks that touch the image border take a general path that
//                loads clamped pixels and replaces the products (and then the responses) of
//                columns outside the image by those of the nearest column inside, which is
//                exactly "window reads clamp on the gradient images" and "NMS reads clamp on
//                the response".  The response arithmetic is the Harris strip kernel's.
#include "harris_strip.hpp"
#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

constexpr int CS_COLS = 240;   // mask columns per strip (60 lanes x 4)

// Interior (strip, row block) pairs: strips s_lo .. s_hi and row blocks b_lo .. b_hi read
// nothing outside the image (columns xm-8 .. xm+247, rows y0-r-2 .. y0+TH+r+1); the rest
// form the border set.  Each set runs as its own launch, so the interior kernel carries no
// border code (and keeps four waves per SIMD at r = 2).
struct Region {
    int nstrips, nblocks;
    int s_lo, s_hi, b_lo, b_hi;   // interior ranges; empty when s_lo > s_hi or b_lo > b_hi
    __host__ __device__ int ni() const { return s_hi >= s_lo ? s_hi - s_lo + 1 : 0; }
    __host__ __device__ int nj() const { return b_hi >= b_lo ? b_hi - b_lo + 1 : 0; }
    __host__ __device__ long long interior() const { return (long long)ni() * nj(); }
    __host__ __device__ long long border() const { return (long long)nstrips * nblocks - interior(); }
    // border work item idx -> (strip, row block): first the row blocks outside b_lo..b_hi
    // across all strips, then the strips outside s_lo..s_hi across the interior row blocks
    __device__ void border_item(int idx, int& strip, int& rb) const {
        if (interior() == 0) {
            strip = idx % nstrips;
            rb = idx / nstrips;
            return;
        }
        const int top = (nblocks - nj()) * nstrips;
        if (idx < top) {
            const int r = idx / nstrips;
            strip = idx % nstrips;
            rb = r < b_lo ? r : r + nj();
        } else {
            const int i2 = idx - top, edge_strips = nstrips - ni();
            const int q = i2 % edge_strips;
            rb = b_lo + i2 / edge_strips;
            strip = q < s_lo ? q : q + ni();
        }
    }
};

// PART 1: the interior set (no clamping anywhere); PART 2: the border set.
template <int RG, int TH, int PART>
__global__ __launch_bounds__(64) void corners_stream(const float* __restrict__ src, size_t sp, uint8_t* __restrict__ M,
                                                     size_t mp, float* __restrict__ resp, size_t rp, int W, int H,
                                                     const float* __restrict__ g, float k, float tau, Region rg_,
                                                     int vec_img, int vec_mask, int vec_resp) {
    constexpr int NW = 2 * RG + 1;   // window taps = ring of pending response rows
    constexpr int D = NW;
    constexpr int NR = TH + 2;       // response rows y0-1 .. y0+TH
    constexpr int K = NR + 2 * RG;   // window rows walked
    const int lane = threadIdx.x;
    int strip, rb;
    if constexpr (PART == 1) {
        strip = rg_.s_lo + (int)(blockIdx.x % (unsigned)rg_.ni());
        rb = rg_.b_lo + (int)(blockIdx.x / (unsigned)rg_.ni());
    } else {
        rg_.border_item((int)blockIdx.x, strip, rb);
    }
    const int y0 = rb * TH;
    const int xm = strip * CS_COLS;
    const int c = xm - 8 + 4 * lane;   // first image column of this lane
    float gw[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) gw[j] = g[j];
    const bool mask_lane = lane >= 2 && lane <= 61;

    auto store_outputs = [&](int y, uint32_t bits, v4f r, bool fast) {
        if (!mask_lane) return;
        uint8_t* mrow = M + (size_t)y * mp + c;
        if (fast && vec_mask) {
            *reinterpret_cast<uint32_t*>(mrow) = bits;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c + q < W) mrow[q] = (uint8_t)(bits >> (8 * q));
        }
        if (resp) {
            float* rrow = reinterpret_cast<float*>(reinterpret_cast<char*>(resp) + (size_t)y * rp) + c;
            if (fast && vec_resp) {
                *reinterpret_cast<v4f*>(rrow) = r;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (c + q < W) rrow[q] = r[q];
            }
        }
    };
    auto response = [&](const v4f (&a)[3]) {
        return mk4(harris_response(a[0].x, a[1].x, a[2].x, k), harris_response(a[0].y, a[1].y, a[2].y, k),
                   harris_response(a[0].z, a[1].z, a[2].z, k), harris_response(a[0].w, a[1].w, a[2].w, k));
    };

    const bool inside_x = vec_img && c - 4 * lane >= 0 && xm - 8 + 256 <= W;
    const bool inside_y = y0 - RG - 2 >= 0 && y0 + TH + RG + 1 <= H - 1;
    if constexpr (PART == 1) {
        if (!(inside_x && inside_y)) return;   // never taken: the host's interior set is exact
        // interior: every read in bounds, nothing clamped.  Window row kk is gradient row
        // y0 - 1 - r + kk, whose Sobel reads image rows y0 - 2 - r + kk + {0, 1, 2}.  The walk
        // is unrolled completely: ring slots and row indices are constants, no branch.
        constexpr int MI = D >= 5 ? D : (D == 3 ? 6 : 5);   // image-row ring
        const char* col = reinterpret_cast<const char*>(src) + (size_t)c * 4;
        auto image_row = [&](int y) { return *reinterpret_cast<const v4f*>(col + (size_t)y * sp); };
        const int ybase = y0 - RG - 2;
        v4f img[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) img[i] = image_row(ybase + i);
        v4f acc[D][3];
#pragma unroll
        for (int u = 0; u < D; ++u) acc[u][0] = acc[u][1] = acc[u][2] = mk4(0.f, 0.f, 0.f, 0.f);
        v4f rr[3];
        static_for<K>([&](auto k_c) {
            constexpr int kk = decltype(k_c)::value;
            v4f qa, qb, qc;
            window_row<RG>(img[kk % MI], img[(kk + 1) % MI], img[(kk + 2) % MI], gw, qa, qb, qc);
            if constexpr (kk + MI <= K + 1) img[kk % MI] = image_row(ybase + kk + MI);
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const int m = kk - j;
                if (m < 0 || m >= NR) continue;
                const int slot = m % D;
                acc[slot][0] += gw[j] * qa;
                acc[slot][1] += gw[j] * qb;
                acc[slot][2] += gw[j] * qc;
            }
            if constexpr (kk >= 2 * RG) {
                constexpr int m = kk - 2 * RG;   // response row y0 - 1 + m is complete
                constexpr int slot = m % D;
                rr[m % 3] = response(acc[slot]);
                acc[slot][0] = acc[slot][1] = acc[slot][2] = mk4(0.f, 0.f, 0.f, 0.f);
                if constexpr (m >= 2) {
                    const uint32_t bits = nms_bits(rr[(m - 2) % 3], rr[(m - 1) % 3], rr[m % 3], tau);
                    store_outputs(y0 + m - 2, bits, rr[(m - 1) % 3], true);
                }
            }
        });
        return;
    } else {
    if (inside_x && inside_y) return;   // never taken: interior items belong to the other launch

    // border strips and row blocks: clamped loads; products and responses of columns outside
    // the image are replaced by those of the nearest column inside
    const bool left = c - 4 * lane < 0;       // strip 0: columns -8 .. -1 are outside
    const bool right = xm - 8 + 256 > W;      // columns >= W are outside
    const int l0 = (0 - (xm - 8)) >> 2;                 // lane holding column 0 (element 0)
    const int l1 = (W - 1 - (xm - 8)) >> 2;             // lane holding column W-1 ...
    const int e1 = (W - 1 - (xm - 8)) & 3;              // ... as element e1
    auto clamp_cols = [&](v4f p) -> v4f {
        if (left) {
            const float v0 = __shfl(p.x, l0 < 0 ? 0 : (l0 > 63 ? 63 : l0));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c + q < 0) p[q] = v0;
        }
        if (right) {
            const float sel = e1 == 0 ? p.x : (e1 == 1 ? p.y : (e1 == 2 ? p.z : p.w));
            const float v1 = __shfl(sel, l1 < 0 ? 0 : (l1 > 63 ? 63 : l1));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c + q >= W) p[q] = v1;
        }
        return p;
    };
    auto image_row = [&](int y) {
        const char* row = reinterpret_cast<const char*>(src) + (size_t)clampi(y, H) * sp;
        if (inside_x) return *reinterpret_cast<const v4f*>(row + (size_t)c * 4);
        v4f v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const float*>(row + (size_t)clampi(c + q, W) * 4);
        return v;
    };
    // window row kk is gradient row clamp(y0 - 1 - r + kk): a repeated gradient row reuses
    // the last products; the image rows around gradient row gr are clamp(gr - 1), gr, clamp(gr + 1)
    auto wrow = [&](int kk) { return clampi(y0 - 1 - RG + kk, H); };
    auto products = [&](v4f ra, v4f rb, v4f rc, v4f& qa, v4f& qb, v4f& qc) {
        v4f pa, pb, pc;
        sobel_products(ra, rb, rc, pa, pb, pc);
        qa = hwin<RG>(clamp_cols(pa), gw);
        qb = hwin<RG>(clamp_cols(pb), gw);
        qc = hwin<RG>(clamp_cols(pc), gw);
    };
    const int g0 = wrow(0);
    v4f ra = image_row(g0 - 1), rb = image_row(g0), rc = image_row(g0 + 1);
    v4f qa, qb, qc;
    products(ra, rb, rc, qa, qb, qc);
    v4f acc[D][3];
#pragma unroll
    for (int u = 0; u < D; ++u) acc[u][0] = acc[u][1] = acc[u][2] = mk4(0.f, 0.f, 0.f, 0.f);
    v4f prev = mk4(0.f, 0.f, 0.f, 0.f), cur = prev;
    for (int kb = 0; kb < K; kb += D) {
        static_for<D>([&](auto u_c) {
            constexpr int u = decltype(u_c)::value;
            const int kk = kb + u;
            if (kk >= K) return;
            if (kk > 0 && wrow(kk) != wrow(kk - 1)) {
                ra = rb;
                rb = rc;
                rc = image_row(wrow(kk) + 1);
                products(ra, rb, rc, qa, qb, qc);
            }
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const int m = kk - j;
                if (m < 0 || m >= NR) continue;
                const int slot = ((u - j) % D + D) % D;
                acc[slot][0] += gw[j] * qa;
                acc[slot][1] += gw[j] * qb;
                acc[slot][2] += gw[j] * qc;
            }
            if (kk >= 2 * RG) {
                constexpr int slot = ((u - 2 * RG) % D + D) % D;
                const int m = kk - 2 * RG;
                const int y = y0 - 1 + m;   // response row just completed
                v4f r = clamp_cols(response(acc[slot]));
                acc[slot][0] = acc[slot][1] = acc[slot][2] = mk4(0.f, 0.f, 0.f, 0.f);
                if (y < 0) return;            // row -1 of the image: row 0 stands in for it
                if (y >= H) r = cur;          // below the image: row H-1 stands in
                // rows y0-1 (m = 0) and y0 (m = 1) fill the ring; row y0 also stands in for
                // row -1 at the top; every later row decides the mask row above it
                const bool fill0 = m == 0, fill1 = m == 1;
                if (!fill0 && !fill1 && y - 1 < H) store_outputs(y - 1, nms_bits(prev, cur, r, tau), cur, false);
                const v4f nprev = fill0 ? r : (fill1 ? (y0 == 0 ? r : prev) : cur);
                const v4f ncur = fill0 ? cur : r;
                prev = nprev;
                cur = ncur;
            }
        });
    }
    }   // PART 2
}

bool supports_stream(const CornersArgs& a) {
    return a.rg >= 0 && a.rg <= 3 && a.nr == 1;
}

template <int RG, int TH>
hipError_t launch_stream_R(const CornersArgs& a) {
    const int vec_img = ((uintptr_t)a.src % 16 == 0) && (a.sp % 16 == 0);
    const int vec_mask = ((uintptr_t)a.M % 4 == 0) && (a.mp % 4 == 0);
    const int vec_resp = a.resp && ((uintptr_t)a.resp % 16 == 0) && (a.rp % 16 == 0);
    Region r{};
    r.nstrips = (a.W + CS_COLS - 1) / CS_COLS;
    r.nblocks = (a.H + TH - 1) / TH;
    if ((long long)r.nstrips * r.nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    // interior strips s: s >= 1 and s * 240 + 248 <= W (columns xm-8 .. xm+247 inside)
    r.s_lo = 1;
    r.s_hi = (vec_img && a.W >= 248) ? (a.W - 248) / CS_COLS : 0;
    // interior row blocks b: b * TH >= r + 2 and b * TH + TH + r + 1 <= H - 1
    r.b_lo = (RG + 2 + TH - 1) / TH;
    const int top = a.H - 2 - RG - TH;
    r.b_hi = top >= 0 ? top / TH : -1;
    if (r.interior() > 0)
        hipLaunchKernelGGL((corners_stream<RG, TH, 1>), dim3((unsigned)r.interior()), dim3(64), 0, a.st, a.src, a.sp,
                           a.M, a.mp, a.resp, a.rp, a.W, a.H, a.g, a.k, a.tau, r, vec_img, vec_mask, vec_resp);
    if (r.border() > 0)
        hipLaunchKernelGGL((corners_stream<RG, TH, 2>), dim3((unsigned)r.border()), dim3(64), 0, a.st, a.src, a.sp,
                           a.M, a.mp, a.resp, a.rp, a.W, a.H, a.g, a.k, a.tau, r, vec_img, vec_mask, vec_resp);
    return hipGetLastError();
}

template <int TH>
hipError_t launch_stream(const CornersArgs& a) {
    switch (a.rg) {
        case 0: return launch_stream_R<0, TH>(a);
        case 1: return launch_stream_R<1, TH>(a);
        case 2: return launch_stream_R<2, TH>(a);
        case 3: return launch_stream_R<3, TH>(a);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ two kernels
// Workspace layout: the response image (W*H floats, only when the caller gives none), then
// the Harris gradient images (only for window radii above the single-pass kernels' range).
size_t resp_bytes(const CornersArgs& a) { return a.resp ? 0 : (((size_t)a.W * a.H * 4 + 255) & ~(size_t)255); }
size_t split_bytes(const CornersArgs& a) { return a.rg > 3 ? harris_workspace(a.W, a.H) : 0; }

bool supports_two_kernel(const CornersArgs& a) {
    const size_t need = resp_bytes(a) + split_bytes(a);
    return need == 0 || (a.ws != nullptr && a.wsb >= need);
}

hipError_t launch_two_kernel(const CornersArgs& a) {
    float* R = a.resp ? a.resp : static_cast<float*>(a.ws);
    const size_t rp = a.resp ? a.rp : (size_t)a.W * 4;
    void* hws = split_bytes(a) ? static_cast<char*>(a.ws) + resp_bytes(a) : nullptr;
    HarrisArgs h{a.src, a.sp, R, rp, a.W, a.H, a.g, a.rg, a.k, hws, split_bytes(a), a.st};
    int hc = 0;
    const Variant<HarrisArgs>* ht = harris_variants(&hc);
    int hv = harris_default(h);
    if (!ht[hv].supports(h)) hv = 0;
    if (!ht[hv].supports(h)) return hipErrorInvalidValue;
    hipError_t e = ht[hv].launch(h);
    if (e != hipSuccess) return e;
    NmsArgs n{R, rp, a.M, a.mp, a.W, a.H, a.nr, a.tau, a.st};
    int nc = 0;
    const Variant<NmsArgs>* nt = nms_variants(&nc);
    int nv = nms_default(n);
    if (!nt[nv].supports(n)) nv = 0;
    return nt[nv].launch(n);
}

const Variant<CornersArgs> kCorners[] = {
    {"two_kernel", supports_two_kernel, launch_two_kernel},
    {"stream_t16", supports_stream, launch_stream<16>},
    {"stream_t24", supports_stream, launch_stream<24>},
    {"stream_t32", supports_stream, launch_stream<32>},
    {"stream_t12", supports_stream, launch_stream<12>},
};

}  // namespace

size_t corners_workspace(int W, int H, int rg) {
    CornersArgs a{};
    a.W = W;
    a.H = H;
    a.rg = rg;
    return resp_bytes(a) + split_bytes(a);
}

const Variant<CornersArgs>* corners_variants(int* count) {
    *count = (int)(sizeof(kCorners) / sizeof(kCorners[0]));
    return kCorners;
}

int corners_default(const CornersArgs& a) { return supports_stream(a) ? 1 : 0; }

}  // namespace icl
