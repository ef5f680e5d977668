// Separable 3-D correlation of volumes (the Image type's 3-D indexing, Section 5; the
// separable passes of the Section 6 benchmark extended by a z pass).
//
//   T1(x,y,z) = sum_i tx[i] V(x+i, y, z)      T2 = sum_j ty[j] T1(x, y+j, z)
//   Y(x,y,z)  = sum_k tz[k] T2(x, y, z+k)     (reads through the boundary condition)
//
// which is the 3-D correlation with taps tz (x) ty (x) tx of the boundary-extended volume.
// A volume is slices of rows: voxel (x, y, z) at base + z * slice_pitch + y * row_pitch +
// x * elem.  Every variant sums each pass in tap order with fmaf from zero, in float32.
//
// Variants
//   plain3p       : three one-voxel-per-thread passes through two float32 workspace volumes.
//   stream_z{TZ}  : one 256-lane work-group per 64 x 16 (x, y) tile and TZ output slices,
//                   walking the TZ + 2r input slices along z: each slice is staged in LDS
//                   (the next one prefetched in registers), its x and y passes run as in the
//                   2-D fused tile, and each lane adds its four voxels into a ring of 2r + 1
//                   pending output slices; the oldest completes and is written.  Every input
//                   voxel is read about (1 + 2r/TZ) times, the intermediates never leave the
//                   chip: 8 B/voxel for float32.
#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "sep_tile.hpp"
#include "tile_stage.hpp"

namespace icl {
namespace {

// ------------------------------------------------------------------ plain three passes
template <class T>
__global__ __launch_bounds__(256) void sep3_x(const void* __restrict__ src, size_t rp, size_t sp,
                                              float* __restrict__ t1, int W, int H, int D,
                                              const float* __restrict__ tx, int r, Border bd) {
    const int x = blockIdx.x * 64 + threadIdx.x % 64;
    const int y = blockIdx.y * 4 + threadIdx.x / 64;
    const int z = blockIdx.z;
    if (x >= W || y >= H) return;
    const size_t row = (size_t)z * sp + (size_t)y * rp;
    float acc = 0.f;
    for (int i = -r; i <= r; ++i) {
        const int xx = x + i;
        const float v = (bd.constant && (xx < 0 || xx >= W)) ? bd.value
                                                             : load_px<T>(src, row + (size_t)clampi(xx, W) * T::size);
        acc = fmaf(tx[i + r], v, acc);
    }
    t1[((size_t)z * H + y) * W + x] = acc;
}

// y pass: rows outside the volume hold sum_i tx[i] c under the constant boundary
__global__ __launch_bounds__(256) void sep3_y(const float* __restrict__ t1, float* __restrict__ t2, int W, int H, int D,
                                              const float* __restrict__ tx, const float* __restrict__ ty, int r,
                                              Border bd) {
    const int x = blockIdx.x * 64 + threadIdx.x % 64;
    const int y = blockIdx.y * 4 + threadIdx.x / 64;
    const int z = blockIdx.z;
    if (x >= W || y >= H) return;
    float c1 = 0.f;
    if (bd.constant)
        for (int i = -r; i <= r; ++i) c1 = fmaf(tx[i + r], bd.value, c1);
    float acc = 0.f;
    for (int j = -r; j <= r; ++j) {
        const int yy = y + j;
        const float v = (bd.constant && (yy < 0 || yy >= H)) ? c1 : t1[((size_t)z * H + clampi(yy, H)) * W + x];
        acc = fmaf(ty[j + r], v, acc);
    }
    t2[((size_t)z * H + y) * W + x] = acc;
}

// z pass: slices outside hold sum_j ty[j] (sum_i tx[i] c)
template <class T>
__global__ __launch_bounds__(256) void sep3_z(const float* __restrict__ t2, void* __restrict__ dst, size_t rp, size_t sp,
                                              int W, int H, int D, const float* __restrict__ tx,
                                              const float* __restrict__ ty, const float* __restrict__ tz, int r,
                                              Border bd) {
    const int x = blockIdx.x * 64 + threadIdx.x % 64;
    const int y = blockIdx.y * 4 + threadIdx.x / 64;
    const int z = blockIdx.z;
    if (x >= W || y >= H) return;
    float c2 = 0.f;
    if (bd.constant) {
        float c1 = 0.f;
        for (int i = -r; i <= r; ++i) c1 = fmaf(tx[i + r], bd.value, c1);
        for (int j = -r; j <= r; ++j) c2 = fmaf(ty[j + r], c1, c2);
    }
    float acc = 0.f;
    for (int k = -r; k <= r; ++k) {
        const int zz = z + k;
        const float v = (bd.constant && (zz < 0 || zz >= D)) ? c2 : t2[((size_t)clampi(zz, D) * H + y) * W + x];
        acc = fmaf(tz[k + r], v, acc);
    }
    store_px<T>(dst, (size_t)z * sp + (size_t)y * rp + (size_t)x * T::size, acc);
}

template <class T>
hipError_t launch_plain_T(const Sep3Args& a) {
    float* t1 = static_cast<float*>(a.ws);
    float* t2 = t1 + (size_t)a.W * a.H * a.D;
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4, a.D);
    hipLaunchKernelGGL(sep3_x<T>, grid, dim3(256), 0, a.st, a.src, a.srp, a.ssp, t1, a.W, a.H, a.D, a.tx, a.r, a.bd);
    hipLaunchKernelGGL(sep3_y, grid, dim3(256), 0, a.st, t1, t2, a.W, a.H, a.D, a.tx, a.ty, a.r, a.bd);
    hipLaunchKernelGGL(sep3_z<T>, grid, dim3(256), 0, a.st, t2, a.dst, a.drp, a.dsp, a.W, a.H, a.D, a.tx, a.ty, a.tz,
                       a.r, a.bd);
    return hipGetLastError();
}

hipError_t launch_plain(const Sep3Args& a) {
    switch (a.dt) {
        case ICL_F32: return launch_plain_T<F32>(a);
        case ICL_F16: return launch_plain_T<F16>(a);
        default: return launch_plain_T<BF16>(a);
    }
}

bool supports_plain(const Sep3Args& a) {
    return a.ws != nullptr && a.wsb >= sep3d_workspace(a.W, a.H, a.D) && a.r >= 0 && a.r <= ICL_MAX_RADIUS_3D &&
           a.D <= 65535;
}

// ------------------------------------------------------------------ z-streaming fused tile
template <class T, int R, int TZ>
__global__ __launch_bounds__(256) void sep3_stream(const void* __restrict__ src, size_t srp, size_t ssp,
                                                   void* __restrict__ dst, size_t drp, size_t dsp, int W, int H,
                                                   int D, const float* __restrict__ tx, const float* __restrict__ ty,
                                                   const float* __restrict__ tz, int tiles_x, int tiles_xy,
                                                   int vec_ok, int vec_out, Border bd) {
    using G = SepTile<R, 16, 1>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR;
    constexpr int KZ = TZ + 2 * R;   // input slices walked
    constexpr int DZ = 2 * R + 1;    // pending output slices
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    float* in_s = lds;
    float* t_s = lds + NR * LW;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(t % (unsigned)tiles_xy);
    const int z0 = (int)(t / (unsigned)tiles_xy) * TZ;
    const int x0 = (tile % tiles_x) * TW, y0 = (tile / tiles_x) * 16;
    Stage<T, NR, LW> st;
    auto load_slice = [&](int kz) {
        const int z = z0 - R + kz;
        if (bd.constant && (z < 0 || z >= D)) {
            st.fill(bd.value);
        } else {
            const char* base = static_cast<const char*>(src) + (size_t)clampi(z, D) * ssp;
            st.load(base, srp, W, H, x0 - RA, y0 - R, vec_ok, bd);
        }
    };
    // lane: columns 4g .. 4g+3 of tile row rg (16 column groups x 16 rows)
    const int g = threadIdx.x % 16, rg = threadIdx.x / 16;
    const int x = x0 + 4 * g, y = y0 + rg;
    float hz[DZ];
#pragma unroll
    for (int k = 0; k < DZ; ++k) hz[k] = tz[k];
    v4f acc[DZ];
#pragma unroll
    for (int k = 0; k < DZ; ++k) acc[k] = mk4(0.f, 0.f, 0.f, 0.f);
    load_slice(0);
    static_for<KZ>([&](auto k_c) {
        constexpr int kz = decltype(k_c)::value;
        __syncthreads();                      // the previous slice's row pass is done with in_s
        st.store(in_s);
        if constexpr (kz + 1 < KZ) load_slice(kz + 1);   // next slice in flight during this one
        __syncthreads();
        sep_row_pass<R, 16, 1>(in_s, t_s, tx);
        __syncthreads();
        // y pass of this lane's four voxels
        v4f v = mk4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j <= 2 * R; ++j) {
            const v4f q = lds4(t_s + (rg + j) * TW + 4 * g);
            const float c = ty[j];
            v.x = fmaf(c, q.x, v.x);
            v.y = fmaf(c, q.y, v.y);
            v.z = fmaf(c, q.z, v.z);
            v.w = fmaf(c, q.w, v.w);
        }
        // z pass: input slice kz feeds output slices kz - k, k = 0 .. 2r
#pragma unroll
        for (int k = 0; k < DZ; ++k) {
            const int m = kz - k;
            if (m < 0 || m >= TZ) continue;
            v4f& a = acc[((kz - k) % DZ + DZ) % DZ];
            a.x = fmaf(hz[k], v.x, a.x);
            a.y = fmaf(hz[k], v.y, a.y);
            a.z = fmaf(hz[k], v.z, a.z);
            a.w = fmaf(hz[k], v.w, a.w);
        }
        if constexpr (kz >= 2 * R) {
            constexpr int m = kz - 2 * R;   // output slice z0 + m is complete
            constexpr int slot = m % DZ;
            const int z = z0 + m;
            if (z < D && y < H) {
                const size_t row = (size_t)z * dsp + (size_t)y * drp;
                const v4f a = acc[slot];
                if (vec_out && x + 4 <= W) {
                    store4<T>(dst, row + (size_t)x * T::size, a);
                } else {
                    if (x < W) store_px<T>(dst, row + (size_t)x * T::size, a.x);
                    if (x + 1 < W) store_px<T>(dst, row + (size_t)(x + 1) * T::size, a.y);
                    if (x + 2 < W) store_px<T>(dst, row + (size_t)(x + 2) * T::size, a.z);
                    if (x + 3 < W) store_px<T>(dst, row + (size_t)(x + 3) * T::size, a.w);
                }
            }
            acc[slot] = mk4(0.f, 0.f, 0.f, 0.f);
        }
    });
}

// Tiles of 64 x TH (TH = 16 or 32) with two staged slices: the next slice goes into the idle
// buffer right after this slice's y pass (its last reader, the previous row pass, finished
// before the barrier that precedes the y pass), so a slice costs two work-group barriers
// instead of three, and the loads of the slice after it are issued then.  A lane takes four
// columns of TH / 16 consecutive rows; the y pass reads each row-pass row once for all of them.
template <class T, int R, int TZ, int TH>
__global__ __launch_bounds__(256) void sep3_stream2(const void* __restrict__ src, size_t srp, size_t ssp,
                                                    void* __restrict__ dst, size_t drp, size_t dsp, int W, int H,
                                                    int D, const float* __restrict__ tx, const float* __restrict__ ty,
                                                    const float* __restrict__ tz, int tiles_x, int tiles_xy,
                                                    int vec_ok, int vec_out, Border bd) {
    using G = SepTile<R, TH, 1>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR, PY = TH / 16;
    constexpr int KZ = TZ + 2 * R;   // input slices walked
    constexpr int DZ = 2 * R + 1;    // pending output slices
    __shared__ __attribute__((aligned(16))) float in_s[2][NR * LW];
    __shared__ __attribute__((aligned(16))) float t_s[NR * TW];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(t % (unsigned)tiles_xy);
    const int z0 = (int)(t / (unsigned)tiles_xy) * TZ;
    const int x0 = (tile % tiles_x) * TW, y0 = (tile / tiles_x) * TH;
    Stage<T, NR, LW> st;
    auto load_slice = [&](int kz) {
        const int z = z0 - R + kz;
        if (bd.constant && (z < 0 || z >= D)) {
            st.fill(bd.value);
        } else {
            const char* base = static_cast<const char*>(src) + (size_t)clampi(z, D) * ssp;
            st.load(base, srp, W, H, x0 - RA, y0 - R, vec_ok, bd);
        }
    };
    const int g = threadIdx.x % 16, rg = threadIdx.x / 16;
    const int x = x0 + 4 * g, ya = y0 + PY * rg;
    float hz[DZ];
#pragma unroll
    for (int k = 0; k < DZ; ++k) hz[k] = tz[k];
    v4f acc[DZ][PY];
#pragma unroll
    for (int k = 0; k < DZ; ++k)
#pragma unroll
        for (int p = 0; p < PY; ++p) acc[k][p] = mk4(0.f, 0.f, 0.f, 0.f);
    load_slice(0);
    st.store(in_s[0]);
    if constexpr (KZ > 1) load_slice(1);
    __syncthreads();
    static_for<KZ>([&](auto k_c) {
        constexpr int kz = decltype(k_c)::value, cur = kz & 1;
        sep_row_pass<R, TH, 1>(in_s[cur], t_s, tx);
        __syncthreads();   // t_s holds this slice's row pass
        // y pass of this lane's PY rows of four voxels
        v4f v[PY];
#pragma unroll
        for (int p = 0; p < PY; ++p) v[p] = mk4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int m = 0; m < PY + 2 * R; ++m) {
            const v4f q = lds4(t_s + (PY * rg + m) * TW + 4 * g);
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                const int j = m - p;
                if (j < 0 || j > 2 * R) continue;
                const float c = ty[j];
                v[p].x = fmaf(c, q.x, v[p].x);
                v[p].y = fmaf(c, q.y, v[p].y);
                v[p].z = fmaf(c, q.z, v[p].z);
                v[p].w = fmaf(c, q.w, v[p].w);
            }
        }
        if constexpr (kz + 1 < KZ) {
            st.store(in_s[cur ^ 1]);
            if constexpr (kz + 2 < KZ) load_slice(kz + 2);   // in flight during the next slice
        }
        // z pass: input slice kz feeds output slices kz - k, k = 0 .. 2r
#pragma unroll
        for (int k = 0; k < DZ; ++k) {
            const int m = kz - k;
            if (m < 0 || m >= TZ) continue;
            const int slot = ((kz - k) % DZ + DZ) % DZ;
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                v4f& a = acc[slot][p];
                a.x = fmaf(hz[k], v[p].x, a.x);
                a.y = fmaf(hz[k], v[p].y, a.y);
                a.z = fmaf(hz[k], v[p].z, a.z);
                a.w = fmaf(hz[k], v[p].w, a.w);
            }
        }
        if constexpr (kz >= 2 * R) {
            constexpr int m = kz - 2 * R;   // output slice z0 + m is complete
            constexpr int slot = m % DZ;
            const int z = z0 + m;
#pragma unroll
            for (int p = 0; p < PY; ++p) {
                const int y = ya + p;
                if (z < D && y < H) {
                    const size_t row = (size_t)z * dsp + (size_t)y * drp;
                    const v4f a = acc[slot][p];
                    if (vec_out && x + 4 <= W) {
                        store4<T>(dst, row + (size_t)x * T::size, a);
                    } else {
                        if (x < W) store_px<T>(dst, row + (size_t)x * T::size, a.x);
                        if (x + 1 < W) store_px<T>(dst, row + (size_t)(x + 1) * T::size, a.y);
                        if (x + 2 < W) store_px<T>(dst, row + (size_t)(x + 2) * T::size, a.z);
                        if (x + 3 < W) store_px<T>(dst, row + (size_t)(x + 3) * T::size, a.w);
                    }
                }
                acc[slot][p] = mk4(0.f, 0.f, 0.f, 0.f);
            }
        }
        __syncthreads();   // the y pass is done with t_s and the next slice is staged
    });
}

template <class T, int R, int TZ, int TH>
hipError_t launch_stream2_TR(const Sep3Args& a) {
    const int tiles_x = (a.W + 63) / 64, tiles_y = (a.H + TH - 1) / TH, zb = (a.D + TZ - 1) / TZ;
    const long long blocks = (long long)tiles_x * tiles_y * zb;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t al = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % al == 0) && (a.srp % al == 0) && (a.ssp % al == 0);
    const int vec_out = ((uintptr_t)a.dst % al == 0) && (a.drp % al == 0) && (a.dsp % al == 0);
    hipLaunchKernelGGL((sep3_stream2<T, R, TZ, TH>), dim3((unsigned)blocks), dim3(256), 0, a.st, a.src, a.srp,
                       a.ssp, a.dst, a.drp, a.dsp, a.W, a.H, a.D, a.tx, a.ty, a.tz, tiles_x, tiles_x * tiles_y,
                       vec_ok, vec_out, a.bd);
    return hipGetLastError();
}

template <class T, int TZ, int TH>
hipError_t launch_stream2_T(const Sep3Args& a) {
    switch (a.r) {
        case 0: return launch_stream2_TR<T, 0, TZ, TH>(a);
        case 1: return launch_stream2_TR<T, 1, TZ, TH>(a);
        case 2: return launch_stream2_TR<T, 2, TZ, TH>(a);
        case 3: return launch_stream2_TR<T, 3, TZ, TH>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TZ, int TH>
hipError_t launch_stream2(const Sep3Args& a) {
    switch (a.dt) {
        case ICL_F32: return launch_stream2_T<F32, TZ, TH>(a);
        case ICL_F16: return launch_stream2_T<F16, TZ, TH>(a);
        default: return launch_stream2_T<BF16, TZ, TH>(a);
    }
}

template <class T, int R, int TZ>
hipError_t launch_stream_TR(const Sep3Args& a) {
    const int tiles_x = (a.W + 63) / 64, tiles_y = (a.H + 15) / 16, zb = (a.D + TZ - 1) / TZ;
    const long long blocks = (long long)tiles_x * tiles_y * zb;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t al = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % al == 0) && (a.srp % al == 0) && (a.ssp % al == 0);
    const int vec_out = ((uintptr_t)a.dst % al == 0) && (a.drp % al == 0) && (a.dsp % al == 0);
    hipLaunchKernelGGL((sep3_stream<T, R, TZ>), dim3((unsigned)blocks), dim3(256), 0, a.st, a.src, a.srp, a.ssp,
                       a.dst, a.drp, a.dsp, a.W, a.H, a.D, a.tx, a.ty, a.tz, tiles_x, tiles_x * tiles_y, vec_ok,
                       vec_out, a.bd);
    return hipGetLastError();
}

template <class T, int TZ>
hipError_t launch_stream_T(const Sep3Args& a) {
    switch (a.r) {
        case 0: return launch_stream_TR<T, 0, TZ>(a);
        case 1: return launch_stream_TR<T, 1, TZ>(a);
        case 2: return launch_stream_TR<T, 2, TZ>(a);
        case 3: return launch_stream_TR<T, 3, TZ>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TZ>
hipError_t launch_stream(const Sep3Args& a) {
    switch (a.dt) {
        case ICL_F32: return launch_stream_T<F32, TZ>(a);
        case ICL_F16: return launch_stream_T<F16, TZ>(a);
        default: return launch_stream_T<BF16, TZ>(a);
    }
}

bool supports_stream(const Sep3Args& a) { return a.r >= 0 && a.r <= 3; }

const Variant<Sep3Args> kSep3[] = {
    {"plain3p", supports_plain, launch_plain},
    {"stream_z16", supports_stream, launch_stream<16>},
    {"stream_z32", supports_stream, launch_stream<32>},
    {"stream_z8", supports_stream, launch_stream<8>},
    {"stream2_z16_h16", supports_stream, launch_stream2<16, 16>},
    {"stream2_z8_h16", supports_stream, launch_stream2<8, 16>},
    {"stream2_z16_h32", supports_stream, launch_stream2<16, 32>},
    {"stream2_z8_h32", supports_stream, launch_stream2<8, 32>},
};

}  // namespace

size_t sep3d_workspace(int W, int H, int D) { return 2 * (size_t)W * (size_t)H * (size_t)D * sizeof(float); }

const Variant<Sep3Args>* sep3d_variants(int* count) {
    *count = (int)(sizeof(kSep3) / sizeof(kSep3[0]));
    return kSep3;
}

// untuned choice: z blocks of 8 slices over 64 x 16 tiles up to r = 1, 64 x 32 tiles beyond
// (the taller tile halves the y halo that a wider window costs)
int sep3d_default(const Sep3Args& a) { return supports_stream(a) ? (a.r <= 1 ? 5 : 7) : 0; }

}  // namespace icl
