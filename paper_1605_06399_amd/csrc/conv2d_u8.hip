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
template <int R> struct U8Strip {
    static constexpr int RA = (R + 3) & ~3;              // halo columns per side (whole words)
    static constexpr int HL = RA / 4;                     // halo lanes per side
    static constexpr int SW = 4 * (64 - 2 * HL);          // output columns per strip
    static constexpr int D = 2 * R + 1;                   // pending output rows
    static constexpr int U = D * ((8 + D - 1) / D);       // unroll: ring slots known at compile time
    static constexpr int Q = 8;                           // input rows in flight ahead
    static constexpr int NW = 1 + 2 * HL;                 // words of a row a lane sees
    static_assert(Q <= U, "prefetch distance must fit the ring");
};

__device__ __forceinline__ uint32_t word_from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t word_from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

template <int R, int TH, bool DOT>
__global__ __launch_bounds__(64) void u8_strip(const uint8_t* __restrict__ src, size_t sp, uint8_t* __restrict__ dst,
                                               size_t dp, int W, int H, const int16_t* __restrict__ taps, int shift,
                                               int nstrips, int vec_in, int vec_out, int cmode, int cval) {
    using G = U8Strip<R>;
    constexpr int RA = G::RA, HL = G::HL, D = G::D, U = G::U, Q = G::Q, NW = G::NW;
    constexpr int K = TH + 2 * R;   // input rows walked
    const int strip = (int)(blockIdx.x % (unsigned)nstrips);
    const int y0 = (int)(blockIdx.x / (unsigned)nstrips) * TH;
    const int lane = threadIdx.x & 63;
    const int c = strip * G::SW - RA + 4 * lane;   // first column of this lane's word
    const bool inside = vec_in && c >= 0 && c + 4 <= W;
    const uint32_t cword = (uint32_t)cval * 0x01010101u;

    auto load_row = [&](int kk) -> uint32_t {
        const int yy = y0 - R + kk;
        if (cmode && (yy < 0 || yy >= H)) return cword;
        const size_t row = (size_t)clampi(yy, H) * sp;
        if (inside) return *reinterpret_cast<const uint32_t*>(src + row + c);
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int xx = c + q;
            const uint32_t b = (cmode && (xx < 0 || xx >= W)) ? (uint32_t)cval : (uint32_t)src[row + clampi(xx, W)];
            v |= b << (8 * q);
        }
        return v;
    };

    // taps: plain values (multiply-add) or packed pairs (dot2): pair t0 + 1 of row j holds
    // (taps[j][t0], taps[j][t0 + 1]) with zero outside 0..2r, t0 = -1 .. 2r
    constexpr int NT = DOT ? D * (D + 1) : D * D;
    int tw[NT];
    {
        const int n = D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if constexpr (DOT) {
#pragma unroll
                for (int t = -1; t < D; ++t) {
                    const int lo = (t >= 0) ? (int)taps[j * n + t] : 0;
                    const int hi = (t + 1 < D) ? (int)taps[j * n + t + 1] : 0;
                    tw[j * (D + 1) + t + 1] = (lo & 0xffff) | (hi << 16);
                }
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) tw[j * D + i] = (int)taps[j * n + i];
            }
        }
    }
    const int bias = shift > 0 ? 1 << (shift - 1) : 0;
    const bool writer = lane >= HL && lane < 64 - HL && c < W;
    const bool wvec = vec_out && c + 4 <= W;

    uint32_t ring[U];
#pragma unroll
    for (int i = 0; i < Q; ++i) ring[i] = i < K ? load_row(i) : 0u;
    int acc[D][4];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[i][p] = 0;

    for (int kb = 0; kb < K; kb += U) {
        static_for<U>([&](auto u_c) {
            constexpr int u = decltype(u_c)::value;
            const int kk = kb + u;
            if (kk >= K) return;
            // the words this lane sees: w[HL] is its own, w[HL - 1] the left neighbour's, ...
            uint32_t wd[NW];
            wd[HL] = ring[u];
            if constexpr (HL >= 1) {
                wd[HL - 1] = word_from_left(wd[HL]);
                wd[HL + 1] = word_from_right(wd[HL]);
            }
            if constexpr (HL >= 2) {
                wd[HL - 2] = word_from_left(wd[HL - 1]);
                wd[HL + 2] = word_from_right(wd[HL + 1]);
            }
            if (kk + Q < K) ring[(u + Q) % U] = load_row(kk + Q);   // that slot's row is consumed
            if constexpr (DOT) {
                // pixel pairs: pair k holds columns (c - RA + 2k, c - RA + 2k + 1) as 16-bit lanes
                constexpr int NP = 2 * NW;
                int pr[NP];
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    pr[k] = (int)__builtin_amdgcn_perm(0u, wd[k / 2], (k & 1) ? 0x0c030c02u : 0x0c010c00u);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int m = kk - j;
                    if (m < 0 || m >= TH) continue;
                    int* a = acc[((u - j) % D + D) % D];
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
#pragma unroll
                        for (int k = 0; k < NP; ++k) {
                            const int t0 = 2 * k - (RA + p - R);   // tap index of the pair's first column
                            if (t0 < -1 || t0 > 2 * R) continue;
                            a[p] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, pr[k]),
                                                          __builtin_bit_cast(short2_t, tw[j * (D + 1) + t0 + 1]),
                                                          a[p], false);
                        }
                    }
                }
            } else {
                int e[4 * NW];
#pragma unroll
                for (int k = 0; k < 4 * NW; ++k) e[k] = (int)((wd[k / 4] >> (8 * (k & 3))) & 0xffu);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int m = kk - j;
                    if (m < 0 || m >= TH) continue;
                    int* a = acc[((u - j) % D + D) % D];
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int i = 0; i < D; ++i) a[p] = __mul24(tw[j * D + i], e[RA - R + p + i]) + a[p];
                }
            }
            if (kk >= 2 * R) {
                constexpr int slot = ((u - 2 * R) % D + D) % D;
                const int y = y0 + kk - 2 * R;
                if (writer && y < H) {
                    uint32_t q[4];
#pragma unroll
                    for (int p = 0; p < 4; ++p) q[p] = (uint32_t)requant(acc[slot][p], shift, bias);
                    uint8_t* o = dst + (size_t)y * dp + c;
                    if (wvec) {
                        *reinterpret_cast<uint32_t*>(o) = q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24);
                    } else {
#pragma unroll
                        for (int p = 0; p < 4; ++p)
                            if (c + p < W) o[p] = (uint8_t)q[p];
                    }
                }
#pragma unroll
                for (int p = 0; p < 4; ++p) acc[slot][p] = 0;
            }
        });
    }
}

template <int R, int TH, bool DOT>
hipError_t launch_strip_R(const U8Args& a) {
    using G = U8Strip<R>;
    const int nstrips = (a.W + G::SW - 1) / G::SW;
    const long long blocks = (long long)nstrips * ((a.H + TH - 1) / TH);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int vec_in = ((uintptr_t)a.src % 4 == 0) && (a.sp % 4 == 0);
    const int vec_out = ((uintptr_t)a.dst % 4 == 0) && (a.dp % 4 == 0);
    hipLaunchKernelGGL((u8_strip<R, TH, DOT>), dim3((unsigned)blocks), dim3(64), 0, a.st, a.src, a.sp, a.dst, a.dp,
                       a.W, a.H, a.taps, a.shift, nstrips, vec_in, vec_out, a.cmode, a.cval);
    return hipGetLastError();
}

constexpr int U8_STRIP_MAX_R = 4;

template <int TH, bool DOT>
hipError_t launch_strip(const U8Args& a) {
    switch (a.r) {
        case 0: return launch_strip_R<0, TH, DOT>(a);
        case 1: return launch_strip_R<1, TH, DOT>(a);
        case 2: return launch_strip_R<2, TH, DOT>(a);
        case 3: return launch_strip_R<3, TH, DOT>(a);
        case 4: return launch_strip_R<4, TH, DOT>(a);
        default: return hipErrorInvalidValue;
    }
}

bool supports_strip(const U8Args& a) { return a.r >= 0 && a.r <= U8_STRIP_MAX_R; }

const Variant<U8Args> kConv2dU8[] = {
    {"plain", supports_plain, launch_plain},
    {"strip_mad_t64", supports_strip, launch_strip<64, false>},
    {"strip_dot_t64", supports_strip, launch_strip<64, true>},
    {"strip_dot_t32", supports_strip, launch_strip<32, true>},
};

}  // namespace

const Variant<U8Args>* conv2d_u8_variants(int* count) {
    *count = (int)(sizeof(kConv2dU8) / sizeof(kConv2dU8[0]));
    return kConv2dU8;
}

int conv2d_u8_default(const U8Args& a) { return supports_strip(a) ? 2 : 0; }

}  // namespace icl
