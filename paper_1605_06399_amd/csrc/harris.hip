// Harris corner response (ImageCL paper, Section 6: Harris corner detection,
// a Sobel kernel (Table 4) followed by a Harris kernel that reads the gradient
// images as Images (Table 5), so window reads clamp on the gradient images).
//
//   Ix = sum s[j] d[i] src(x+i, y+j),  Iy = sum d[j] s[i] src(x+i, y+j)
//        s = (1,2,1), d = (-1,0,1)
//   Sxx = sum_{j,i} g[j] g[i] Ix^2(x+i, y+j)   (Syy from Iy^2, Sxy from Ix*Iy)
//   R   = Sxx*Syy - Sxy^2 - k*(Sxx+Syy)^2
//
// Variants
//   plain_split   : the paper's two kernels with naive mapping: Sobel writes Ix, Iy
//                   (float32, workspace), the Harris kernel reads them with a
//                   clamped 2-D window loop.  16 B/px of HBM beyond in/out.
//   fused_t{TH}   : one pass per 64 x TH tile.  The image tile with a (1 + rg) halo
//                   is staged in LDS; gradients are evaluated at the clamped
//                   positions of the (64+2rg) x (TH+2rg) gradient region (which is
//                   exactly "window reads clamp on the gradient image"), their
//                   products go to LDS, and the separable window runs as a row pass
//                   into LDS and a column pass in registers.  8 B/px of HBM.
//   stream_t{TH}  : one wave per 248-column strip and TH rows, walking down the rows
//                   with everything in registers (one float4 image load per lane and
//                   row, neighbour columns by DPP lane shifts, rings of prefetched image
//                   rows and of pending output rows); the 4-column left band and the
//                   right remainder run through the tile kernel.  16-byte aligned rows.
#include "harris_strip.hpp"
#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

// ------------------------------------------------------------------ plain split
__global__ __launch_bounds__(256) void sobel_plain(const float* __restrict__ src, size_t sp, float* __restrict__ ix,
                                                   float* __restrict__ iy, int W, int H) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    const float s[3] = {1.f, 2.f, 1.f}, d[3] = {-1.f, 0.f, 1.f};
    float gx = 0.f, gy = 0.f;
    for (int j = -1; j <= 1; ++j) {
        const float* row = reinterpret_cast<const float*>(reinterpret_cast<const char*>(src) +
                                                          (size_t)clampi(y + j, H) * sp);
        for (int i = -1; i <= 1; ++i) {
            const float p = row[clampi(x + i, W)];
            gx += s[j + 1] * d[i + 1] * p;
            gy += d[j + 1] * s[i + 1] * p;
        }
    }
    ix[(size_t)y * W + x] = gx;
    iy[(size_t)y * W + x] = gy;
}

__global__ __launch_bounds__(256) void harris_window_plain(const float* __restrict__ ix, const float* __restrict__ iy,
                                                           float* __restrict__ resp, size_t rp, int W, int H,
                                                           const float* __restrict__ g, int rg, float k) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    float a = 0.f, b = 0.f, c = 0.f;
    for (int j = -rg; j <= rg; ++j)
        for (int i = -rg; i <= rg; ++i) {
            const size_t q = (size_t)clampi(y + j, H) * W + clampi(x + i, W);
            const float w = g[j + rg] * g[i + rg];
            const float gx = ix[q], gy = iy[q];
            a += w * gx * gx;
            b += w * gy * gy;
            c += w * gx * gy;
        }
    float* out = reinterpret_cast<float*>(reinterpret_cast<char*>(resp) + (size_t)y * rp);
    out[x] = harris_response(a, b, c, k);
}

hipError_t launch_plain(const HarrisArgs& a) {
    float* ix = static_cast<float*>(a.ws);
    float* iy = ix + (size_t)a.W * a.H;
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
    hipLaunchKernelGGL(sobel_plain, grid, dim3(256), 0, a.st, a.src, a.sp, ix, iy, a.W, a.H);
    hipLaunchKernelGGL(harris_window_plain, grid, dim3(256), 0, a.st, ix, iy, a.resp, a.rp, a.W, a.H, a.g, a.rg, a.k);
    return hipGetLastError();
}

bool supports_plain(const HarrisArgs& a) {
    return a.ws != nullptr && a.wsb >= harris_workspace(a.W, a.H) && a.rg >= 0 && a.rg <= ICL_MAX_WINDOW_RADIUS;
}

// ------------------------------------------------------------------ fused tile
template <int RG, int TH> struct HTile {
    static constexpr int TW = 64;
    static constexpr int HX = RG + 1;                 // image halo rows / cols needed
    static constexpr int HXA = (HX + 3) & ~3;         // column halo rounded to float4
    static constexpr int IW = TW + 2 * HXA;           // staged image row length
    static constexpr int IR = TH + 2 * HX;            // staged image rows
    static constexpr int GW = TW + 2 * RG;            // gradient region
    static constexpr int GH = TH + 2 * RG;
    static constexpr int PY = TH / 4;
    static constexpr int REGION1 = (IR * IW > 3 * GH * TW) ? IR * IW : 3 * GH * TW;   // image, later h
    static constexpr int LDS_FLOATS = REGION1 + 3 * GH * GW;
};

// Tile columns come in two bands: the first n0 start at 0 (step TW) and write columns
// below xl; the rest start at xr (step TW) and write columns below W.  The full image is
// n0 = tiles_x, xl = W.
template <int RG, int TH>
__global__ __launch_bounds__(256) void harris_fused(const float* __restrict__ src, size_t sp, float* __restrict__ resp,
                                                    size_t rp, int W, int H, const float* __restrict__ g, float k,
                                                    int tiles_x, int n0, int xl, int xr, int vec_ok) {
    using G = HTile<RG, TH>;
    constexpr int TW = G::TW, HX = G::HX, HXA = G::HXA, IW = G::IW, IR = G::IR, GW = G::GW, GH = G::GH,
                  PY = G::PY;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    float* img = lds;                      // [IR][IW], dead after the gradient stage
    float* hs = lds;                       // [3][GH][TW] row-pass sums (reuses img)
    float* abc = lds + G::REGION1;         // [3][GH][GW] products Ix^2, Iy^2, Ix*Iy
    const int tid = threadIdx.x;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)tiles_x);
    const int x0 = tx < n0 ? tx * TW : xr + (tx - n0) * TW;
    const int xe = tx < n0 ? xl : W;       // columns this tile may write
    const int y0 = (int)(t / (unsigned)tiles_x) * TH;

    // 1. stage image rows y0-HX .. y0+TH+HX-1, columns x0-HXA .. x0+TW+HXA-1 (clamped)
    // every load is issued before the LDS writes (a load-then-write loop would wait on each)
    if (vec_ok && x0 - HXA >= 0 && x0 + TW + HXA <= W) {
        constexpr int C4 = IW / 4, NCH = IR * C4, PER = (NCH + 255) / 256;
        v4f v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int y = clampi(y0 - HX + rr, H);
            v[i] = *reinterpret_cast<const v4f*>(reinterpret_cast<const char*>(src) + (size_t)y * sp +
                                                 (size_t)(x0 - HXA + 4 * c4) * 4);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NCH % 256 != 0 && idx >= NCH) break;
            const int rr = idx / C4, c4 = idx - rr * C4;
            lds4(&img[rr * IW + 4 * c4], v[i]);
        }
    } else {
        constexpr int NE = IR * IW, PER = (NE + 255) / 256;
        float v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NE % 256 != 0 && idx >= NE) break;
            const int rr = idx / IW, c = idx - rr * IW;
            const int y = clampi(y0 - HX + rr, H);
            const int x = clampi(x0 - HXA + c, W);
            v[i] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(src) + (size_t)y * sp + (size_t)x * 4);
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (NE % 256 != 0 && idx >= NE) break;
            img[idx] = v[i];
        }
    }
    __syncthreads();

    // 2. gradients at the clamped position of every gradient-region pixel, then products
    for (int idx = tid; idx < GH * GW; idx += 256) {
        const int gr = idx / GW, gc = idx - gr * GW;
        const int cy = clampi(y0 - RG + gr, H), cx = clampi(x0 - RG + gc, W);
        const float* p = &img[(cy - (y0 - HX)) * IW + (cx - (x0 - HXA))];
        const float a00 = p[-IW - 1], a01 = p[-IW], a02 = p[-IW + 1];
        const float a10 = p[-1], a12 = p[1];
        const float a20 = p[IW - 1], a21 = p[IW], a22 = p[IW + 1];
        const float ix = (a02 - a00) + 2.f * (a12 - a10) + (a22 - a20);
        const float iy = (a20 - a00) + 2.f * (a21 - a01) + (a22 - a02);
        abc[idx] = ix * ix;
        abc[GH * GW + idx] = iy * iy;
        abc[2 * GH * GW + idx] = ix * iy;
    }
    __syncthreads();

    // 3. window row pass over the three product images
    for (int idx = tid; idx < GH * TW; idx += 256) {
        const int gr = idx / TW, c = idx - gr * TW;
        float sa = 0.f, sb = 0.f, sc = 0.f;
#pragma unroll
        for (int i = 0; i <= 2 * RG; ++i) {
            const float w = g[i];
            const int q = gr * GW + c + i;
            sa = fmaf(w, abc[q], sa);
            sb = fmaf(w, abc[GH * GW + q], sb);
            sc = fmaf(w, abc[2 * GH * GW + q], sc);
        }
        hs[idx] = sa;
        hs[GH * TW + idx] = sb;
        hs[2 * GH * TW + idx] = sc;
    }
    __syncthreads();

    // 4. window column pass and response: lane owns column lx, rows ly*PY .. ly*PY+PY-1
    const int lx = tid & 63, ly = tid >> 6;
    float va[PY + 2 * RG], vb[PY + 2 * RG], vc[PY + 2 * RG];
#pragma unroll
    for (int m = 0; m < PY + 2 * RG; ++m) {
        const int q = (ly * PY + m) * TW + lx;
        va[m] = hs[q];
        vb[m] = hs[GH * TW + q];
        vc[m] = hs[2 * GH * TW + q];
    }
    const int x = x0 + lx;
#pragma unroll
    for (int py = 0; py < PY; ++py) {
        float sa = 0.f, sb = 0.f, sc = 0.f;
#pragma unroll
        for (int j = 0; j <= 2 * RG; ++j) {
            const float w = g[j];
            sa = fmaf(w, va[py + j], sa);
            sb = fmaf(w, vb[py + j], sb);
            sc = fmaf(w, vc[py + j], sc);
        }
        const int y = y0 + ly * PY + py;
        if (x < xe && y < H)
            reinterpret_cast<float*>(reinterpret_cast<char*>(resp) + (size_t)y * rp)[x] = harris_response(sa, sb, sc, k);
    }
}

// Tile kernel over the bands [0, xl) and [xr, W) (xl = W: the whole image).
template <int RG, int TH>
hipError_t launch_fused_bands(const HarrisArgs& a, int xl, int xr) {
    using G = HTile<RG, TH>;
    const int n0 = (xl + G::TW - 1) / G::TW;
    const int n1 = xl >= a.W ? 0 : (a.W - xr + G::TW - 1) / G::TW;
    const int tiles_x = n0 + n1;
    const int tiles_y = (a.H + TH - 1) / TH;
    const int vec_ok = ((uintptr_t)a.src % 16 == 0) && (a.sp % 16 == 0);
    hipLaunchKernelGGL((harris_fused<RG, TH>), dim3(tiles_x * tiles_y), dim3(256), 0, a.st, a.src, a.sp, a.resp, a.rp,
                       a.W, a.H, a.g, a.k, tiles_x, n0, xl, xr, vec_ok);
    return hipGetLastError();
}

template <int RG, int TH>
hipError_t launch_fused_R(const HarrisArgs& a) {
    return launch_fused_bands<RG, TH>(a, a.W, a.W);
}

// ------------------------------------------------------------------ streaming strips
// One wave per strip of HS_COLS output columns and TH rows.  Lane l holds the four image
// columns xs-4+4l .. xs-1+4l; lanes 1..62 own the strip's outputs, lanes 0 and 63 only
// supply the left and right halo (3 columns suffice: Sobel 1 + window radius <= 3 = 4),
// so every read of the strip is inside the image and nothing is clamped in x.  The wave
// walks down the clamped window rows: per row it loads one float4 of the image per lane
// (prefetched D rows ahead), forms the vertical Sobel parts from the last three image
// rows, gets the neighbouring columns by DPP lane shifts, forms the three products and
// their horizontal window sum, and adds that row into a ring of D = 2r+1 pending output
// rows; the oldest completes and is written each step.  No LDS tile, no barrier.
constexpr int HS_COLS = 248;   // output columns per strip (62 lanes x 4)
constexpr int HS_XL = 4;       // left border band (the strips start here), done by the tile kernel

// One wave per work-group (the register allocation of a 64-lane launch bound keeps the
// working set at four waves per SIMD without spills).
template <int RG, int TH>
__global__ __launch_bounds__(64) void harris_stream(const float* __restrict__ src, size_t sp, float* __restrict__ resp,
                                                    size_t rp, int H, const float* __restrict__ g, float k,
                                                    int nstrips) {
    constexpr int NW = 2 * RG + 1;   // window taps = length of the ring of pending output rows
    constexpr int K = TH + 2 * RG;   // window rows walked per strip
    constexpr int D = NW;
    const int lane = threadIdx.x;
    const int strip = (int)(blockIdx.x % (unsigned)nstrips);
    const int y0 = (int)(blockIdx.x / (unsigned)nstrips) * TH;
    const int c = HS_XL + strip * HS_COLS - 4 + 4 * lane;
    const char* col = reinterpret_cast<const char*>(src) + (size_t)c * 4;
    auto image_row = [&](int y) { return *reinterpret_cast<const v4f*>(col + (size_t)y * sp); };
    float gw[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) gw[j] = g[j];
    v4f acc[D][3];
#pragma unroll
    for (int u = 0; u < D; ++u) acc[u][0] = acc[u][1] = acc[u][2] = mk4(0.f, 0.f, 0.f, 0.f);
    const bool writer = lane >= 1 && lane <= 62;
    char* out_col = reinterpret_cast<char*>(resp) + (size_t)c * 4;

    // window row kk (phase u = kk mod D of the ring) feeds output rows kk - j; output row
    // kk - 2r is then complete and is written
    auto accumulate_emit = [&](int kk, auto u_c, v4f qa, v4f qb, v4f qc) {
        constexpr int u = decltype(u_c)::value;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int m = kk - j;
            if (m < 0 || m >= TH) continue;
            const int slot = ((u - j) % D + D) % D;
            acc[slot][0] += gw[j] * qa;
            acc[slot][1] += gw[j] * qb;
            acc[slot][2] += gw[j] * qc;
        }
        if (kk >= 2 * RG) {
            constexpr int slot = ((u - 2 * RG) % D + D) % D;
            const int y = y0 + kk - 2 * RG;
            const v4f sa = acc[slot][0], sb = acc[slot][1], sc = acc[slot][2];
            if (writer && y < H)
                *reinterpret_cast<v4f*>(out_col + (size_t)y * rp) =
                    mk4(harris_response(sa.x, sb.x, sc.x, k), harris_response(sa.y, sb.y, sc.y, k),
                        harris_response(sa.z, sb.z, sc.z, k), harris_response(sa.w, sb.w, sc.w, k));
            acc[slot][0] = acc[slot][1] = acc[slot][2] = mk4(0.f, 0.f, 0.f, 0.f);
        }
    };

    if (y0 - RG - 1 >= 0 && y0 + TH + RG <= H - 1) {
        // interior row block: window row kk is gradient row y0 - r + kk, whose Sobel reads
        // image rows y0 - r - 1 + kk + {0, 1, 2}; those come from a ring of M image rows
        // (image row i of the block in slot i mod M), each loaded M - 2 steps before use
        // The walk is unrolled completely (TH is small), so every ring slot, row range and
        // prefetch bound is a constant and the steady state has no branch.
        constexpr int M = D >= 5 ? D : (D == 3 ? 6 : 5);
        const int ybase = y0 - RG - 1;
        v4f img[M];
#pragma unroll
        for (int i = 0; i < M; ++i) img[i] = image_row(ybase + i);
        static_for<K>([&](auto k_c) {
            constexpr int kk = decltype(k_c)::value;
            v4f qa, qb, qc;
            window_row<RG>(img[kk % M], img[(kk + 1) % M], img[(kk + 2) % M], gw, qa, qb, qc);
            if constexpr (kk + M <= K + 1) img[kk % M] = image_row(ybase + kk + M);
            accumulate_emit(kk, std::integral_constant<int, kk % D>{}, qa, qb, qc);
        });
        return;
    }

    // row block at the top or bottom edge: window rows clamp to the gradient image, so a
    // repeated gradient row reuses the last products and the image rows around gradient row
    // g are clamp(g - 1), g, clamp(g + 1)
    auto wrow = [&](int kk) { return clampi(y0 - RG + kk, H); };
    const int g0 = wrow(0);
    v4f ra = image_row(clampi(g0 - 1, H)), rb = image_row(g0), rc = image_row(clampi(g0 + 1, H));
    v4f qa, qb, qc;
    window_row<RG>(ra, rb, rc, gw, qa, qb, qc);
    for (int kb = 0; kb < K; kb += D) {
        static_for<D>([&](auto u_c) {
            constexpr int u = decltype(u_c)::value;
            const int kk = kb + u;
            if (kk >= K) return;
            if (kk > 0 && wrow(kk) != wrow(kk - 1)) {
                ra = rb;
                rb = rc;
                rc = image_row(clampi(wrow(kk) + 1, H));
                window_row<RG>(ra, rb, rc, gw, qa, qb, qc);
            }
            accumulate_emit(kk, u_c, qa, qb, qc);
        });
    }
}

bool supports_stream(const HarrisArgs& a) {
    return a.rg >= 0 && a.rg <= 3 && a.W >= HS_XL + HS_COLS + 4 && (uintptr_t)a.src % 16 == 0 && a.sp % 16 == 0 &&
           (uintptr_t)a.resp % 16 == 0 && a.rp % 16 == 0;
}

template <int RG, int TH>
hipError_t launch_stream_R(const HarrisArgs& a) {
    const int nstrips = (a.W - HS_XL - 4) / HS_COLS;
    const int xr = HS_XL + nstrips * HS_COLS;
    const int rows = (a.H + TH - 1) / TH;
    hipLaunchKernelGGL((harris_stream<RG, TH>), dim3((unsigned)(nstrips * rows)), dim3(64), 0, a.st, a.src, a.sp,
                       a.resp, a.rp, a.H, a.g, a.k, nstrips);
    // the two border bands with the tile kernel
    return launch_fused_bands<RG, 16>(a, HS_XL, xr);
}

template <int TH>
hipError_t launch_stream(const HarrisArgs& a) {
    switch (a.rg) {
        case 0: return launch_stream_R<0, TH>(a);
        case 1: return launch_stream_R<1, TH>(a);
        case 2: return launch_stream_R<2, TH>(a);
        case 3: return launch_stream_R<3, TH>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TH>
hipError_t launch_fused(const HarrisArgs& a) {
    switch (a.rg) {
        case 0: return launch_fused_R<0, TH>(a);
        case 1: return launch_fused_R<1, TH>(a);
        case 2: return launch_fused_R<2, TH>(a);
        case 3: return launch_fused_R<3, TH>(a);
        default: return hipErrorInvalidValue;
    }
}

bool supports_fused(const HarrisArgs& a) { return a.rg >= 0 && a.rg <= 3; }

const Variant<HarrisArgs> kHarris[] = {
    {"plain_split", supports_plain, launch_plain},
    {"fused_t16", supports_fused, launch_fused<16>},
    {"fused_t32", supports_fused, launch_fused<32>},
    {"fused_t8", supports_fused, launch_fused<8>},
    {"stream_t64", supports_stream, launch_stream<64>},
    {"stream_t32", supports_stream, launch_stream<32>},
    {"stream_t16", supports_stream, launch_stream<16>},
    {"stream_t12", supports_stream, launch_stream<12>},
};

}  // namespace

size_t harris_workspace(int W, int H) { return 2 * (size_t)W * (size_t)H * sizeof(float); }

const Variant<HarrisArgs>* harris_variants(int* count) {
    *count = (int)(sizeof(kHarris) / sizeof(kHarris[0]));
    return kHarris;
}

// strip variant with 32-row blocks where the rows allow it, else the 64 x 16 tile kernel
int harris_default(const HarrisArgs& a) { return supports_stream(a) ? 5 : supports_fused(a) ? 1 : 0; }

}  // namespace icl
