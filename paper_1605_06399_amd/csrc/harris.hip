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
#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

__device__ __forceinline__ float harris_response(float sxx, float syy, float sxy, float k) {
    const float tr = sxx + syy;
    return sxx * syy - sxy * sxy - k * tr * tr;
}

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

template <int RG, int TH>
__global__ __launch_bounds__(256) void harris_fused(const float* __restrict__ src, size_t sp, float* __restrict__ resp,
                                                    size_t rp, int W, int H, const float* __restrict__ g, float k,
                                                    int tiles_x, int vec_ok) {
    using G = HTile<RG, TH>;
    constexpr int TW = G::TW, HX = G::HX, HXA = G::HXA, IW = G::IW, IR = G::IR, GW = G::GW, GH = G::GH,
                  PY = G::PY;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    float* img = lds;                      // [IR][IW], dead after the gradient stage
    float* hs = lds;                       // [3][GH][TW] row-pass sums (reuses img)
    float* abc = lds + G::REGION1;         // [3][GH][GW] products Ix^2, Iy^2, Ix*Iy
    const int tid = threadIdx.x;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (int)(t % (unsigned)tiles_x) * TW;
    const int y0 = (int)(t / (unsigned)tiles_x) * TH;

    // 1. stage image rows y0-HX .. y0+TH+HX-1, columns x0-HXA .. x0+TW+HXA-1 (clamped)
    if (vec_ok && x0 - HXA >= 0 && x0 + TW + HXA <= W) {
        constexpr int C4 = IW / 4;
        for (int idx = tid; idx < IR * C4; idx += 256) {
            const int rr = idx / C4, c4 = idx - rr * C4;
            const int y = clampi(y0 - HX + rr, H);
            lds4(&img[rr * IW + 4 * c4], *reinterpret_cast<const v4f*>(
                reinterpret_cast<const char*>(src) + (size_t)y * sp + (size_t)(x0 - HXA + 4 * c4) * 4));
        }
    } else {
        for (int idx = tid; idx < IR * IW; idx += 256) {
            const int rr = idx / IW, c = idx - rr * IW;
            const int y = clampi(y0 - HX + rr, H);
            const int x = clampi(x0 - HXA + c, W);
            img[rr * IW + c] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(src) +
                                                               (size_t)y * sp + (size_t)x * 4);
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
        if (x < W && y < H)
            reinterpret_cast<float*>(reinterpret_cast<char*>(resp) + (size_t)y * rp)[x] = harris_response(sa, sb, sc, k);
    }
}

template <int RG, int TH>
hipError_t launch_fused_R(const HarrisArgs& a) {
    using G = HTile<RG, TH>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + TH - 1) / TH;
    const int vec_ok = ((uintptr_t)a.src % 16 == 0) && (a.sp % 16 == 0);
    hipLaunchKernelGGL((harris_fused<RG, TH>), dim3(tiles_x * tiles_y), dim3(256), 0, a.st, a.src, a.sp, a.resp, a.rp,
                       a.W, a.H, a.g, a.k, tiles_x, vec_ok);
    return hipGetLastError();
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
};

}  // namespace

size_t harris_workspace(int W, int H) { return 2 * (size_t)W * (size_t)H * sizeof(float); }

const Variant<HarrisArgs>* harris_variants(int* count) {
    *count = (int)(sizeof(kHarris) / sizeof(kHarris[0]));
    return kHarris;
}

int harris_default(const HarrisArgs& a) { return supports_fused(a) ? 1 : 0; }

}  // namespace icl
