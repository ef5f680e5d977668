// Non-maximum suppression with threshold, the last stage of corner detection
// (thresholding the Harris response to a corner mask; the paper's Harris
// benchmark stops at the response, so the rule is the library's definition):
//
//   mask(x,y) = 1  iff  R(x,y) > tau  and  R(x,y) >= R(clamp(x+i), clamp(y+j))
//                        for all |i|, |j| <= r,
//             = 0  otherwise.
//
// With clamped reads an outside neighbour is an inside pixel that is already in
// the neighbourhood (or the centre itself), so the rule equals "ignore pixels
// outside the image".  Comparisons are exact float32 comparisons; NaN fails.
//
// Variants
//   plain      : one thread per pixel, 16x16 work-groups, clamped reads, runtime radius.
//   row4       : one lane per 4 consecutive pixels of a row (r = 1): three aligned
//                float4 row loads plus the two flanking pixels, one 32-bit store of
//                four mask bytes; clamps only on edge lanes.
#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

__global__ __launch_bounds__(256) void nms_plain(const float* __restrict__ R, size_t rp, uint8_t* __restrict__ M,
                                                 size_t mp, int W, int H, int r, float tau) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    auto at = [&](int xx, int yy) {
        return reinterpret_cast<const float*>(reinterpret_cast<const char*>(R) + (size_t)yy * rp)[xx];
    };
    const float c = at(x, y);
    bool keep = c > tau;
    for (int j = -r; j <= r && keep; ++j)
        for (int i = -r; i <= r; ++i)
            if (!(c >= at(clampi(x + i, W), clampi(y + j, H)))) { keep = false; break; }
    M[(size_t)y * mp + x] = keep ? 1 : 0;
}

hipError_t launch_plain(const NmsArgs& a) {
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
    hipLaunchKernelGGL(nms_plain, grid, dim3(256), 0, a.st, a.R, a.rp, a.M, a.mp, a.W, a.H, a.r, a.tau);
    return hipGetLastError();
}

bool supports_plain(const NmsArgs& a) { return a.r >= 1 && a.r <= ICL_MAX_NMS_RADIUS; }

// ------------------------------------------------------------------ four pixels per lane, r = 1
__device__ __forceinline__ void row6(const float* __restrict__ row, int x, int W, bool interior, float v[6]) {
    if (interior) {
        const v4f m = *reinterpret_cast<const v4f*>(row + x);
        v[0] = row[x - 1]; v[1] = m.x; v[2] = m.y; v[3] = m.z; v[4] = m.w; v[5] = row[x + 4];
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = row[clampi(x - 1 + k, W)];
    }
}

__global__ __launch_bounds__(256) void nms_row4(const float* __restrict__ R, size_t rp, uint8_t* __restrict__ M,
                                                size_t mp, int W, int H, float tau, int groups_x, int vec_ok) {
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    const int y = (int)(gid / groups_x);
    const int x = (int)(gid - (long long)y * groups_x) * 4;
    if (y >= H) return;
    const bool interior = vec_ok && x >= 1 && x + 5 <= W;
    float a[6], b[6], c[6];
    const char* base = reinterpret_cast<const char*>(R);
    row6(reinterpret_cast<const float*>(base + (size_t)clampi(y - 1, H) * rp), x, W, interior, a);
    row6(reinterpret_cast<const float*>(base + (size_t)y * rp), x, W, interior, b);
    row6(reinterpret_cast<const float*>(base + (size_t)clampi(y + 1, H) * rp), x, W, interior, c);
    uint32_t bits = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float v = b[p + 1];
        const bool keep = v > tau && v >= a[p] && v >= a[p + 1] && v >= a[p + 2] && v >= b[p] && v >= b[p + 2] &&
                          v >= c[p] && v >= c[p + 1] && v >= c[p + 2];
        bits |= (keep ? 1u : 0u) << (8 * p);
    }
    uint8_t* out = M + (size_t)y * mp + x;
    if (vec_ok && x + 4 <= W) {
        *reinterpret_cast<uint32_t*>(out) = bits;
    } else {
        for (int p = 0; p < 4 && x + p < W; ++p) out[p] = (uint8_t)((bits >> (8 * p)) & 1u);
    }
}

hipError_t launch_row4(const NmsArgs& a) {
    const int groups_x = (a.W + 3) / 4;
    const long long n = (long long)groups_x * a.H;
    const int vec_ok = ((uintptr_t)a.R % 16 == 0) && (a.rp % 16 == 0) && ((uintptr_t)a.M % 4 == 0) && (a.mp % 4 == 0);
    hipLaunchKernelGGL(nms_row4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, a.st, a.R, a.rp, a.M, a.mp, a.W, a.H,
                       a.tau, groups_x, vec_ok);
    return hipGetLastError();
}

bool supports_row4(const NmsArgs& a) { return a.r == 1; }

const Variant<NmsArgs> kNms[] = {
    {"plain", supports_plain, launch_plain},
    {"row4", supports_row4, launch_row4},
};

}  // namespace

const Variant<NmsArgs>* nms_variants(int* count) {
    *count = (int)(sizeof(kNms) / sizeof(kNms[0]));
    return kNms;
}

int nms_default(const NmsArgs& a) { return supports_row4(a) ? 1 : 0; }

}  // namespace icl
