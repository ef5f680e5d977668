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
//   stream_t{TH}: one wave per 248-column strip and TH rows (r = 1): every response row
//                loaded once, the 3 x 3 neighbourhood from registers and DPP lane shifts;
//                the border bands run through row4.  16-byte aligned response rows.
//   stream_a_t{TH}: one wave per 256-column strip at a multiple of 256 and TH rows (r = 1):
//                all 64 lanes own outputs, aligned 1 KiB row reads and 256-byte mask writes,
//                the two outside columns as broadcast values; columns right of the last whole
//                strip run through row4.  _sm: strip-major wave order.
#include "harris_strip.hpp"
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

// Column groups come in two bands: the first n0 groups start at column 0 and write columns
// below xl, the rest start at xr and write columns below W (the whole image: n0 = all, xl = W).
__global__ __launch_bounds__(256) void nms_row4(const float* __restrict__ R, size_t rp, uint8_t* __restrict__ M,
                                                size_t mp, int W, int H, float tau, int groups_x, int n0, int xl,
                                                int xr, int vec_ok) {
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    const int y = (int)(gid / groups_x);
    const int gx = (int)(gid - (long long)y * groups_x);
    const int x = gx < n0 ? 4 * gx : xr + 4 * (gx - n0);
    const int xe = gx < n0 ? xl : W;
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
        const bool keep = (v > tau) & (v >= a[p]) & (v >= a[p + 1]) & (v >= a[p + 2]) & (v >= b[p]) & (v >= b[p + 2]) &
                          (v >= c[p]) & (v >= c[p + 1]) & (v >= c[p + 2]);
        bits |= (keep ? 1u : 0u) << (8 * p);
    }
    uint8_t* out = M + (size_t)y * mp + x;
    if (vec_ok && x + 4 <= xe) {
        *reinterpret_cast<uint32_t*>(out) = bits;
    } else {
        for (int p = 0; p < 4 && x + p < xe; ++p) out[p] = (uint8_t)((bits >> (8 * p)) & 1u);
    }
}

// Row kernel over the bands [0, xl) and [xr, W) (xl = W: the whole image).
hipError_t launch_row4_bands(const NmsArgs& a, int xl, int xr) {
    const int n0 = (xl + 3) / 4;
    const int n1 = xl >= a.W ? 0 : (a.W - xr + 3) / 4;
    const int groups_x = n0 + n1;
    const long long n = (long long)groups_x * a.H;
    const int vec_ok = ((uintptr_t)a.R % 16 == 0) && (a.rp % 16 == 0) && ((uintptr_t)a.M % 4 == 0) && (a.mp % 4 == 0);
    hipLaunchKernelGGL(nms_row4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, a.st, a.R, a.rp, a.M, a.mp, a.W, a.H,
                       a.tau, groups_x, n0, xl, xr, vec_ok);
    return hipGetLastError();
}

hipError_t launch_row4(const NmsArgs& a) { return launch_row4_bands(a, a.W, a.W); }

bool supports_row4(const NmsArgs& a) { return a.r == 1; }

// ------------------------------------------------------------------ strips, r = 1
// One wave per strip of NS_COLS columns and TH rows: lane l holds the four columns
// xs-4+4l .. xs-1+4l of the response rows, lanes 1..62 own the outputs and lanes 0 and 63
// only supply the neighbouring column, so no read of a strip is clamped in x.  The wave
// walks down the rows holding the rows above, at and below the output row in registers
// (each row loaded once, prefetched through a ring), gets the left and right neighbours by
// DPP lane shifts and writes the four mask bytes of a lane as one 32-bit store.  The left
// 4 columns and the right remainder (under 252 columns) run through the row kernel.
constexpr int NS_COLS = 248;
constexpr int NS_XL = 4;

// Four independent strip waves per work-group (wave w of group b is strip wave 4b + w).
template <int TH>
__global__ __launch_bounds__(256) void nms_stream(const float* __restrict__ R, size_t rp, uint8_t* __restrict__ M,
                                                  size_t mp, int H, float tau, int nstrips, int nwaves) {
    const int lane = threadIdx.x & 63;
    const int wv = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wv >= nwaves) return;   // no barrier in this kernel: a wave may leave early
    const int strip = wv % nstrips;
    const int y0 = (wv / nstrips) * TH;
    const int c = NS_XL + strip * NS_COLS - 4 + 4 * lane;
    const char* col = reinterpret_cast<const char*>(R) + (size_t)c * 4;
    auto row = [&](int y) { return *reinterpret_cast<const v4f*>(col + (size_t)y * rp); };
    const bool writer = lane >= 1 && lane <= 62;
    uint8_t* out_col = M + c;
    if (y0 >= 1 && y0 + TH <= H - 1) {
        // interior: output row m reads rows y0 - 1 + m + {0, 1, 2}, from a ring of RING rows
        // (row i of the block in slot i mod RING), each loaded RING - 2 rows before use
        // completely unrolled (TH is small): constant ring slots and bounds, no branch
        constexpr int RING = 8;
        const int ybase = y0 - 1;
        v4f ring[RING];
#pragma unroll
        for (int i = 0; i < RING; ++i) ring[i] = row(ybase + i);
        static_for<TH>([&](auto m_c) {
            constexpr int m = decltype(m_c)::value;
            const uint32_t bits = nms_bits(ring[m % RING], ring[(m + 1) % RING], ring[(m + 2) % RING], tau);
            if constexpr (m + RING <= TH + 1) ring[m % RING] = row(ybase + m + RING);
            if (writer) *reinterpret_cast<uint32_t*>(out_col + (size_t)(y0 + m) * mp) = bits;
        });
        return;
    }
    // top or bottom block: rows clamp at the image edge
    for (int m = 0; m < TH; ++m) {
        const int y = y0 + m;
        if (y >= H) break;
        const uint32_t bits = nms_bits(row(clampi(y - 1, H)), row(y), row(clampi(y + 1, H)), tau);
        if (writer) *reinterpret_cast<uint32_t*>(out_col + (size_t)y * mp) = bits;
    }
}

bool supports_stream(const NmsArgs& a) {
    return a.r == 1 && a.W >= NS_XL + NS_COLS + 4 && (uintptr_t)a.R % 16 == 0 && a.rp % 16 == 0 &&
           (uintptr_t)a.M % 4 == 0 && a.mp % 4 == 0;
}

template <int TH>
hipError_t launch_stream(const NmsArgs& a) {
    const int nstrips = (a.W - NS_XL - 4) / NS_COLS;
    const int xr = NS_XL + nstrips * NS_COLS;
    const int rows = (a.H + TH - 1) / TH;
    const int nwaves = nstrips * rows;
    hipLaunchKernelGGL(nms_stream<TH>, dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, a.st, a.R, a.rp, a.M, a.mp,
                       a.H, a.tau, nstrips, nwaves);
    return launch_row4_bands(a, NS_XL, xr);
}

// ------------------------------------------------------------------ aligned strips, r = 1
// One wave per 256-column strip starting at a multiple of 256 and TH rows: every lane owns
// four output columns, so each response row is one aligned 1 KiB read and each mask row one
// aligned 256-byte write.  The two columns just outside the strip (its neighbours' edge
// pixels, clamped at the image border) are read as one broadcast value each and replace the
// DPP shift's missing neighbour in lanes 0 and 63.  Columns right of the last whole strip
// run through the row kernel.
__device__ __forceinline__ uint32_t nms_bits_edges(v4f a, v4f b, v4f c, float al_e, float ar_e, float bl_e, float br_e,
                                                   float cl_e, float cr_e, float tau) {
    const float al = lane_from_left_or(a.w, al_e), ar = lane_from_right_or(a.x, ar_e);
    const float bl = lane_from_left_or(b.w, bl_e), br = lane_from_right_or(b.x, br_e);
    const float cl = lane_from_left_or(c.w, cl_e), cr = lane_from_right_or(c.x, cr_e);
    const float ea[6] = {al, a.x, a.y, a.z, a.w, ar};
    const float eb[6] = {bl, b.x, b.y, b.z, b.w, br};
    const float ec[6] = {cl, c.x, c.y, c.z, c.w, cr};
    uint32_t bits = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float v = eb[p + 1];
        const bool keep = (v > tau) & (v >= ea[p]) & (v >= ea[p + 1]) & (v >= ea[p + 2]) & (v >= eb[p]) &
                          (v >= eb[p + 2]) & (v >= ec[p]) & (v >= ec[p + 1]) & (v >= ec[p + 2]);
        bits |= (keep ? 1u : 0u) << (8 * p);
    }
    return bits;
}

// SM: strip-major wave order after the XCD remap (the four waves of a work-group and the
// work-groups an XCD runs together are consecutive row blocks of one strip, so the row
// above and below a block come from that XCD's L2); otherwise row-major (the waves running
// together read whole image rows).
template <int TH, bool SM>
__global__ __launch_bounds__(256) void nms_stream_a(const float* __restrict__ R, size_t rp, uint8_t* __restrict__ M,
                                                    size_t mp, int W, int H, float tau, int nstrips, int nwaves) {
    const int lane = threadIdx.x & 63;
    int strip, y0;
    if constexpr (SM) {
        const int wv = (int)xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6);
        if (wv >= nwaves) return;   // no barrier in this kernel: a wave may leave early
        const int nrb = nwaves / nstrips;
        strip = wv / nrb;
        y0 = (wv - strip * nrb) * TH;
    } else {
        const int wv = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
        if (wv >= nwaves) return;
        strip = wv % nstrips;
        y0 = (wv / nstrips) * TH;
    }
    const int x0 = strip * 256;
    const int xl = x0 > 0 ? x0 - 1 : 0, xr = x0 + 256 < W ? x0 + 256 : W - 1;
    const char* base = reinterpret_cast<const char*>(R);
    auto row = [&](int y) { return *reinterpret_cast<const v4f*>(base + (size_t)y * rp + (size_t)(x0 + 4 * lane) * 4); };
    auto px = [&](int y, int x) { return *reinterpret_cast<const float*>(base + (size_t)y * rp + (size_t)x * 4); };
    uint8_t* out = M + x0 + 4 * lane;
    if (y0 >= 1 && y0 + TH <= H - 1) {
        // interior: output row m reads rows y0 - 1 + m + {0, 1, 2} from a ring of RING rows
        // (row i of the block in slot i mod RING), each loaded RING - 2 rows before use; a
        // block of fewer than RING - 2 rows loads only its TH + 2 rows (the rows after them
        // may lie past the image)
        constexpr int RING = 8, NPRE = TH + 2 < RING ? TH + 2 : RING;
        const int ybase = y0 - 1;
        v4f ring[RING];
        float el[RING], er[RING];
#pragma unroll
        for (int i = 0; i < NPRE; ++i) {
            ring[i] = row(ybase + i);
            el[i] = px(ybase + i, xl);
            er[i] = px(ybase + i, xr);
        }
        static_for<TH>([&](auto m_c) {
            constexpr int m = decltype(m_c)::value, a = m % RING, b = (m + 1) % RING, c = (m + 2) % RING;
            const uint32_t bits = nms_bits_edges(ring[a], ring[b], ring[c], el[a], er[a], el[b], er[b], el[c], er[c], tau);
            if constexpr (m + RING <= TH + 1) {
                ring[a] = row(ybase + m + RING);
                el[a] = px(ybase + m + RING, xl);
                er[a] = px(ybase + m + RING, xr);
            }
            *reinterpret_cast<uint32_t*>(out + (size_t)(y0 + m) * mp) = bits;
        });
        return;
    }
    // top or bottom block: rows clamp at the image edge
    for (int m = 0; m < TH; ++m) {
        const int y = y0 + m;
        if (y >= H) break;
        const int ya = clampi(y - 1, H), yc = clampi(y + 1, H);
        const uint32_t bits = nms_bits_edges(row(ya), row(y), row(yc), px(ya, xl), px(ya, xr), px(y, xl), px(y, xr),
                                             px(yc, xl), px(yc, xr), tau);
        *reinterpret_cast<uint32_t*>(out + (size_t)y * mp) = bits;
    }
}

bool supports_stream_a(const NmsArgs& a) {
    return a.r == 1 && a.W >= 256 && (uintptr_t)a.R % 16 == 0 && a.rp % 16 == 0 && (uintptr_t)a.M % 4 == 0 &&
           a.mp % 4 == 0;
}

template <int TH, bool SM>
hipError_t launch_stream_a(const NmsArgs& a) {
    const int nstrips = a.W / 256;
    const int rows = (a.H + TH - 1) / TH;
    const long long nwaves = (long long)nstrips * rows;
    if (nwaves > 0x7ffffff0LL) return hipErrorInvalidValue;
    const long long blocks = (nwaves + 3) / 4;
    hipLaunchKernelGGL((nms_stream_a<TH, SM>), dim3(SM ? grid_pad8(blocks) : (unsigned)blocks), dim3(256), 0, a.st,
                       a.R, a.rp, a.M, a.mp, a.W, a.H, a.tau, nstrips, (int)nwaves);
    if (nstrips * 256 < a.W) return launch_row4_bands(a, 0, nstrips * 256);
    return hipGetLastError();
}

const Variant<NmsArgs> kNms[] = {
    {"plain", supports_plain, launch_plain},
    {"row4", supports_row4, launch_row4},
    {"stream_t64", supports_stream, launch_stream<64>},
    {"stream_t32", supports_stream, launch_stream<32>},
    {"stream_a_t64", supports_stream_a, launch_stream_a<64, false>},
    {"stream_a_t32", supports_stream_a, launch_stream_a<32, false>},
    {"stream_a_t16", supports_stream_a, launch_stream_a<16, false>},
    {"stream_a_t8", supports_stream_a, launch_stream_a<8, false>},
    {"stream_a_t4", supports_stream_a, launch_stream_a<4, false>},
    {"stream_a_t32_sm", supports_stream_a, launch_stream_a<32, true>},
    {"stream_a_t16_sm", supports_stream_a, launch_stream_a<16, true>},
};

}  // namespace

const Variant<NmsArgs>* nms_variants(int* count) {
    *count = (int)(sizeof(kNms) / sizeof(kNms[0]));
    return kNms;
}

int nms_default(const NmsArgs& a) { return supports_stream(a) ? 2 : supports_row4(a) ? 1 : 0; }

}  // namespace icl
