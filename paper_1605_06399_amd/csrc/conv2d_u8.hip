// 2-D correlation of unsigned char images with signed 16-bit taps (the non-separable
// convolution benchmark of Section 6 runs on unsigned char pixels).
//
//   S(x,y) = sum_{j,i=-r..r} taps[(j+r)(2r+1) + (i+r)] * src(x+i, y+j)     (exact, int32)
//   dst(x,y) = min(max((S + 2^(shift-1)) >> shift, 0), 255)   (bias 0 when shift = 0)
//
// The sum is exact in 32-bit integers for r <= 7 (|S| <= 225 * 2^15 * 255 < 2^31), so
// every variant returns the same bytes whatever its order of accumulation.
//
// Variants:
//   plain         : one thread per pixel, direct loads, one multiply-add per tap.
//   strip_mad_t64 : one wave per strip of 4 * (64 - 2 ceil(r/4)) columns and 64 rows.
//                   Lane l holds the four pixels (one 32-bit word) of its columns of every
//                   input row it walks; the horizontal neighbours arrive through DPP lane
//                   shifts; a ring of 2r+1 pending output rows takes each input row's
//                   contribution to every output row it touches, so every input byte is
//                   loaded once per strip.  One 24-bit multiply-add per tap and pixel.
//   strip_dot_t64 / strip_dot_t32 : the same walk, with the pixels widened to pairs of
//                   16-bit lanes and the taps pre-packed into pairs, so one v_dot2_i32_i16
//                   takes two taps: r + 1 dot products per pixel and tap row instead of
//                   2r + 1 multiply-adds.
#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int requant(int s, int shift, int bias) { return min(max((s + bias) >> shift, 0), 255); }

// Output byte of a sum that already holds the rounding bias.  The empty asm hides the
// clamp's range from the compiler, so the four bytes are packed with full 32-bit
// shifts and ors: otherwise gfx950 code generation may fuse shift, saturation and
// packing into v_ashr_pk_u8_i32, which writes only the low half of its destination
// while the or that follows assumes the upper half is zero.
__device__ __forceinline__ uint32_t out_byte(int s, int shift) {
    int q = min(max(s >> shift, 0), 255);
    asm volatile("" : "+v"(q));
    return (uint32_t)q;
}

// ------------------------------------------------------------------ plain
__global__ __launch_bounds__(256) void u8_plain(const uint8_t* __restrict__ src, size_t sp, uint8_t* __restrict__ dst,
                                                size_t dp, int W, int H, const int16_t* __restrict__ taps, int r,
                                                int shift, int cmode, int cval) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    const int n = 2 * r + 1;
    int acc = 0;
    for (int j = -r; j <= r; ++j) {
        const bool yout = y + j < 0 || y + j >= H;
        const size_t row = (size_t)clampi(y + j, H) * sp;
        for (int i = -r; i <= r; ++i) {
            const bool out = cmode && (yout || x + i < 0 || x + i >= W);
            const int p = out ? cval : (int)src[row + clampi(x + i, W)];
            acc += (int)taps[(j + r) * n + (i + r)] * p;
        }
    }
    dst[(size_t)y * dp + x] = (uint8_t)requant(acc, shift, shift > 0 ? 1 << (shift - 1) : 0);
}

hipError_t launch_plain(const U8Args& a) {
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
    hipLaunchKernelGGL(u8_plain, grid, dim3(256), 0, a.st, a.src, a.sp, a.dst, a.dp, a.W, a.H, a.taps, a.r,
                       a.shift, a.cmode, a.cval);
    return hipGetLastError();
}

bool supports_plain(const U8Args& a) { return a.r >= 0 && a.r <= ICL_MAX_U8_RADIUS; }

// ------------------------------------------------------------------ register-streaming strips
// A lane holds PX consecutive pixels (PX / 4 words) of every input row its wave walks.  For
// r >= 1 the first and last lane of the wave only supply the horizontal halo (r <= 4
// columns: one word of each neighbour lane), so a strip has PX * 62 output columns; for
// r = 0 every lane writes.
template <int R, int PX> struct U8Strip {
    static_assert(R >= 0 && R <= 4, "strip kernels cover radii 0..4");
    static constexpr int HL = R > 0 ? 1 : 0;               // halo lanes per side
    static constexpr int NWL = PX / 4;                     // words a lane loads per row
    static constexpr int SW = PX * (64 - 2 * HL);          // output columns per strip
    static constexpr int OFF = HL ? 4 : 0;                 // window column of the lane's first pixel
    static constexpr int NW = NWL + 2 * HL;                // words of a row a lane sees
    static constexpr int D = 2 * R + 1;                    // tap rows
    static constexpr int Q = 8;                            // input rows in flight ahead
};

__device__ __forceinline__ uint32_t word_from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t word_from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

template <int PX> struct RowWords { uint32_t w[PX / 4]; };

// One strip of TH output rows, all K = TH + 2r input rows unrolled so that every ring slot,
// accumulator row and output condition is known at compile time.
//   EDGE = false: every word of every lane lies inside the image, and source and destination
//                 rows are PX-byte aligned (the interior strips): one vector load and one
//                 vector store per lane and row.
//   EDGE = true : any strip; each byte is read through the boundary condition and
//                 written only if it lies inside the image.
// Per input row: the neighbour lanes' boundary words arrive by DPP lane shifts, the
// pixels are widened to 16-bit pairs (v_perm), and each output pixel takes, per tap row,
// r + 1 packed dot products against tap pairs (taps[j][t], taps[j][t+1]) aligned to its
// column parity.  The sums start from the rounding bias, so the output is
// med3(acc >> shift, 0, 255).
// QD > 0: QD input rows in flight ahead instead of the default eight (the _q16 variants hold
// all but a few rows of a short strip in flight from its start).
template <int R, int TH, int PX, bool EDGE, int QD = 0>
__device__ __forceinline__ void u8_strip_body(const uint8_t* __restrict__ src, size_t sp, uint8_t* __restrict__ dst,
                                              size_t dp, int W, int H, const int* __restrict__ tw, int shift,
                                              int bias, int c, int y0, int cmode, int cval) {
    using G = U8Strip<R, PX>;
    constexpr int HL = G::HL, NWL = G::NWL, NW = G::NW, OFF = G::OFF, D = G::D;
    constexpr int K = TH + 2 * R;
    constexpr int QQ = QD > 0 ? QD : G::Q;
    constexpr int Q = K < QQ ? K : QQ;
    const int lane = threadIdx.x & 63;
    const uint32_t cword = (uint32_t)cval * 0x01010101u;

    auto load_row = [&](int kk) -> RowWords<PX> {
        RowWords<PX> v;
        const int yy = y0 - R + kk;
        if (cmode && (yy < 0 || yy >= H)) {
#pragma unroll
            for (int q = 0; q < NWL; ++q) v.w[q] = cword;
            return v;
        }
        const uint8_t* row = src + (size_t)clampi(yy, H) * sp;
        if constexpr (!EDGE) {
            if constexpr (PX == 8) {
                const uint2 t = *reinterpret_cast<const uint2*>(row + c);
                v.w[0] = t.x;
                v.w[1] = t.y;
            } else {
                v.w[0] = *reinterpret_cast<const uint32_t*>(row + c);
            }
        } else {
#pragma unroll
            for (int q = 0; q < NWL; ++q) {
                uint32_t word = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int xx = c + 4 * q + b;
                    const uint32_t px =
                        (cmode && (xx < 0 || xx >= W)) ? (uint32_t)cval : (uint32_t)row[clampi(xx, W)];
                    word |= px << (8 * b);
                }
                v.w[q] = word;
            }
        }
        return v;
    };

    const bool writer = lane >= HL && lane < 64 - HL && (!EDGE || c < W);
    RowWords<PX> ring[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) ring[i] = load_row(i);
    int acc[D][PX];

    static_for<K>([&](auto kk_c) {
        constexpr int kk = decltype(kk_c)::value;
        uint32_t wd[NW];
#pragma unroll
        for (int q = 0; q < NWL; ++q) wd[HL + q] = ring[kk % Q].w[q];
        if constexpr (kk + Q < K) ring[kk % Q] = load_row(kk + Q);   // slot consumed: refill
        if constexpr (HL == 1) {
            wd[0] = word_from_left(wd[NWL]);          // left lane's last word
            wd[NWL + 1] = word_from_right(wd[1]);     // right lane's first word
        }
        // pixel pairs: pair k holds window columns (2k, 2k + 1) as 16-bit lanes
        constexpr int NP = 2 * NW;
        int pr[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            pr[k] = (int)__builtin_amdgcn_perm(0u, wd[k / 2], (k & 1) ? 0x0c030c02u : 0x0c010c00u);
        static_for<D>([&](auto j_c) {
            constexpr int j = decltype(j_c)::value;
            constexpr int m = kk - j;   // output row this input row feeds through tap row j
            if constexpr (m >= 0 && m < TH) {
                int* a = acc[m % D];
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    if constexpr (j == 0) a[p] = bias;   // first contribution to output row m
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const int t0 = 2 * k - (OFF + p - R);   // tap index of the pair's first column
                        if (t0 < -1 || t0 > 2 * R) continue;
                        a[p] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, pr[k]),
                                                      __builtin_bit_cast(short2_t, tw[j * (D + 1) + t0 + 1]), a[p],
                                                      false);
                    }
                }
            }
        });
        if constexpr (kk >= 2 * R) {
            constexpr int m = kk - 2 * R;   // output row complete
            const int y = y0 + m;
            if (writer && y < H) {
                uint32_t o4[NWL];
#pragma unroll
                for (int q = 0; q < NWL; ++q) {
                    uint32_t b[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) b[t] = out_byte(acc[m % D][4 * q + t], shift);
                    o4[q] = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
                }
                uint8_t* o = dst + (size_t)y * dp + c;
                if constexpr (!EDGE) {
                    if constexpr (PX == 8)
                        *reinterpret_cast<uint2*>(o) = make_uint2(o4[0], o4[1]);
                    else
                        *reinterpret_cast<uint32_t*>(o) = o4[0];
                } else {
#pragma unroll
                    for (int p = 0; p < PX; ++p)
                        if (c + p < W) o[p] = (uint8_t)(o4[p / 4] >> (8 * (p & 3)));
                }
            }
        }
    });
}

template <int R, int TH, int PX, int QD = 0>
__global__ __launch_bounds__(64) void u8_strip(const uint8_t* __restrict__ src, size_t sp, uint8_t* __restrict__ dst,
                                               size_t dp, int W, int H, const int16_t* __restrict__ taps, int shift,
                                               int nstrips, int vec, int cmode, int cval) {
    using G = U8Strip<R, PX>;
    constexpr int D = G::D;
    const int strip = (int)(blockIdx.x % (unsigned)nstrips);
    const int y0 = (int)(blockIdx.x / (unsigned)nstrips) * TH;
    const int lane = threadIdx.x & 63;
    const int x0 = strip * G::SW - G::HL * PX;   // first column of lane 0
    const int c = x0 + PX * lane;

    // tap pairs: entry t0 + 1 of row j holds (taps[j][t0], taps[j][t0 + 1]), zero outside
    // 0..2r, for t0 = -1 .. 2r
    int tw[D * (D + 1)];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
        for (int t = -1; t < D; ++t) {
            const int lo = (t >= 0) ? (int)taps[j * D + t] : 0;
            const int hi = (t + 1 < D) ? (int)taps[j * D + t + 1] : 0;
            tw[j * (D + 1) + t + 1] = (lo & 0xffff) | (hi << 16);
        }
    const int bias = shift > 0 ? 1 << (shift - 1) : 0;
    const bool interior = vec && x0 >= 0 && x0 + 64 * PX <= W;
    if (interior)
        u8_strip_body<R, TH, PX, false, QD>(src, sp, dst, dp, W, H, tw, shift, bias, c, y0, cmode, cval);
    else
        u8_strip_body<R, TH, PX, true, QD>(src, sp, dst, dp, W, H, tw, shift, bias, c, y0, cmode, cval);
}

template <int R, int TH, int PX, int QD = 0>
hipError_t launch_strip_R(const U8Args& a) {
    using G = U8Strip<R, PX>;
    const int nstrips = (a.W + G::SW - 1) / G::SW;
    const long long blocks = (long long)nstrips * ((a.H + TH - 1) / TH);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    // interior strips use PX-byte vector loads and stores: both images' rows must be aligned
    const int vec = ((uintptr_t)a.src % PX == 0) && (a.sp % PX == 0) && ((uintptr_t)a.dst % PX == 0) &&
                    (a.dp % PX == 0);
    hipLaunchKernelGGL((u8_strip<R, TH, PX, QD>), dim3((unsigned)blocks), dim3(64), 0, a.st, a.src, a.sp, a.dst, a.dp,
                       a.W, a.H, a.taps, a.shift, nstrips, vec, a.cmode, a.cval);
    return hipGetLastError();
}

constexpr int U8_STRIP_MAX_R = 4;

template <int TH, int PX, int QD = 0>
hipError_t launch_strip(const U8Args& a) {
    switch (a.r) {
        case 0: return launch_strip_R<0, TH, PX, QD>(a);
        case 1: return launch_strip_R<1, TH, PX, QD>(a);
        case 2: return launch_strip_R<2, TH, PX, QD>(a);
        case 3: return launch_strip_R<3, TH, PX, QD>(a);
        case 4: return launch_strip_R<4, TH, PX, QD>(a);
        default: return hipErrorInvalidValue;
    }
}

bool supports_strip(const U8Args& a) { return a.r >= 0 && a.r <= U8_STRIP_MAX_R; }

const Variant<U8Args> kConv2dU8[] = {
    {"plain", supports_plain, launch_plain},
    {"strip_p4_t16", supports_strip, launch_strip<16, 4>},
    {"strip_p4_t32", supports_strip, launch_strip<32, 4>},
    {"strip_p8_t16", supports_strip, launch_strip<16, 8>},
    {"strip_p8_t32", supports_strip, launch_strip<32, 8>},
    {"strip_p4_t24", supports_strip, launch_strip<24, 4>},
    {"strip_p4_t16_q16", supports_strip, launch_strip<16, 4, 16>},
    {"strip_p4_t12_q16", supports_strip, launch_strip<12, 4, 16>},
};

}  // namespace

const Variant<U8Args>* conv2d_u8_variants(int* count) {
    *count = (int)(sizeof(kConv2dU8) / sizeof(kConv2dU8[0]));
    return kConv2dU8;
}

int conv2d_u8_default(const U8Args& a) { return supports_strip(a) ? 1 : 0; }

}  // namespace icl
