// Separable convolution with clamped reads (ImageCL paper, Section 6:
// separable convolution benchmark, row kernel R and column kernel C, Table 2).
//
//   T(x,y)   = sum_i tx[i+r] * src(clamp(x+i), y)
//   dst(x,y) = sum_j ty[j+r] * T(x, clamp(y+j))
//
// Variants
//   plain2p           : the paper's naive code generation, twice: one thread per
//                       pixel, 16x16 work-groups, clamp on every read, runtime tap
//                       loop; the row pass writes a float32 intermediate to HBM.
//   fused_t{TH}_c{CX} : one pass.  A work-group owns a 64*CX x TH output tile,
//                       stages the (TH+2r) x (64*CX+2*RA) input rows it needs in
//                       LDS (float4 loads for interior tiles), runs the row pass
//                       four columns per lane into a second LDS tile, and the
//                       column pass from LDS with TH/4 rows per lane.  The
//                       intermediate never leaves the CU (the fusion the paper's
//                       discussion credits for Halide's win).  CX = 2 gives each
//                       lane two columns 64 apart (interleaved within the
//                       work-group, Fig. 4c), keeping stores coalesced.
//   pers_t{TH}_c{CX}  : the fused tile body in a persistent grid that prefetches the
//                       next tile into registers while computing the current one.
//   fused_img_t{TH}_c{CX}: the fused tile staged through one buffer descriptor per row,
//                       whose hardware range check supplies the constant-0 boundary (the
//                       stand-in for the paper's image-memory candidate; see below), one pixel
//                       per lane; fused_img4: four pixels per lane.
//   colwalk_s{SEG}    : persistent work-groups walk 64-column strips down SEG-row segments,
//                       staging and row-passing each input row once (sep_colwalk.hpp).
//   strip_t{TH}       : one wave per strip of 256 - 8*ceil(r/4) output columns and TH
//                       rows, walking down the rows with both passes in registers:
//                       horizontal neighbours by DPP lane shifts, a ring of 2r+1
//                       pending output rows for the vertical pass, prefetched input
//                       rows.  No LDS, no barrier; the same float32 expression per
//                       output as the tile variants.
#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "sep_colwalk.hpp"
#include "sep_strip.hpp"
#include "sep_tile.hpp"
#include "tile_stage.hpp"

namespace icl {
namespace {

// ------------------------------------------------------------------ plain two-pass
template <class T>
__global__ __launch_bounds__(256) void sep_row_plain(const void* __restrict__ src, size_t sp,
                                                     float* __restrict__ tmp, int W, int H,
                                                     const float* __restrict__ tx, int r, Border bd) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    float acc = 0.f;
    for (int i = -r; i <= r; ++i) {
        const int xx = x + i;
        const float v = (bd.constant && (xx < 0 || xx >= W))
                            ? bd.value
                            : load_px<T>(src, (size_t)y * sp + (size_t)clampi(xx, W) * T::size);
        acc += tx[i + r] * v;
    }
    tmp[(size_t)y * W + x] = acc;
}

// With a constant boundary a row outside the image is the constant everywhere, so its row
// pass is sum_i tx[i] * c (summed in the row pass's order).
template <class T>
__global__ __launch_bounds__(256) void sep_col_plain(const float* __restrict__ tmp, void* __restrict__ dst,
                                                     size_t dp, int W, int H, const float* __restrict__ tx,
                                                     const float* __restrict__ ty, int r, Border bd) {
    const int x = blockIdx.x * 16 + threadIdx.x % 16;
    const int y = blockIdx.y * 16 + threadIdx.x / 16;
    if (x >= W || y >= H) return;
    float outside = 0.f;
    if (bd.constant)
        for (int i = -r; i <= r; ++i) outside = fmaf(tx[i + r], bd.value, outside);
    float acc = 0.f;
    for (int j = -r; j <= r; ++j) {
        const int yy = y + j;
        const float v = (bd.constant && (yy < 0 || yy >= H)) ? outside : tmp[(size_t)clampi(yy, H) * W + x];
        acc += ty[j + r] * v;
    }
    store_px<T>(dst, (size_t)y * dp + (size_t)x * T::size, acc);
}

template <class T>
hipError_t launch_plain_T(const SepArgs& a) {
    float* tmp = static_cast<float*>(a.ws);
    dim3 grid((a.W + 15) / 16, (a.H + 15) / 16);
    hipLaunchKernelGGL(sep_row_plain<T>, grid, dim3(256), 0, a.st, a.src, a.sp, tmp, a.W, a.H, a.tx, a.r, a.bd);
    hipLaunchKernelGGL(sep_col_plain<T>, grid, dim3(256), 0, a.st, tmp, a.dst, a.dp, a.W, a.H, a.tx, a.ty, a.r,
                       a.bd);
    return hipGetLastError();
}

hipError_t launch_plain(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_plain_T<F32>(a);
        case ICL_F16: return launch_plain_T<F16>(a);
        default: return launch_plain_T<BF16>(a);
    }
}

bool supports_plain(const SepArgs& a) {
    return a.ws != nullptr && a.wsb >= sep_workspace(a.W, a.H) && a.r >= 0 && a.r <= ICL_MAX_RADIUS;
}

}  // namespace

namespace {

template <class T, int R, int TH, int CX>
__global__ __launch_bounds__(256) void sep_fused(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                 size_t dp, int W, int H, const float* __restrict__ tx,
                                                 const float* __restrict__ ty, int tiles_x, int vec_ok, int vec_out,
                                                 Border bd) {
    using G = SepTile<R, TH, CX>;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (int)(t % (unsigned)tiles_x) * G::TW;
    const int y0 = (int)(t / (unsigned)tiles_x) * TH;
    const bool vec = vec_ok && x0 - G::RA >= 0 && x0 + G::TW + G::RA <= W;
    sep_tile_body<T, R, TH, CX>(src, sp, dst, dp, W, H, tx, ty, x0, y0, vec, vec_out, lds, bd);
}

template <class T, int R, int TH, int CX>
hipError_t launch_fused_TR(const SepArgs& a) {
    using G = SepTile<R, TH, CX>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + TH - 1) / TH;
    const size_t vec_align = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % vec_align == 0) && (a.sp % vec_align == 0);
    const int vec_out = ((uintptr_t)a.dst % vec_align == 0) && (a.dp % vec_align == 0);
    hipLaunchKernelGGL((sep_fused<T, R, TH, CX>), dim3(tiles_x * tiles_y), dim3(256), 0, a.st, a.src, a.sp,
                       a.dst, a.dp, a.W, a.H, a.tx, a.ty, tiles_x, vec_ok, vec_out, a.bd);
    return hipGetLastError();
}

template <class T, int TH, int CX>
hipError_t launch_fused_T(const SepArgs& a) {
    switch (a.r) {
        case 0: return launch_fused_TR<T, 0, TH, CX>(a);
        case 1: return launch_fused_TR<T, 1, TH, CX>(a);
        case 2: return launch_fused_TR<T, 2, TH, CX>(a);
        case 3: return launch_fused_TR<T, 3, TH, CX>(a);
        case 4: return launch_fused_TR<T, 4, TH, CX>(a);
        case 5: return launch_fused_TR<T, 5, TH, CX>(a);
        case 6: return launch_fused_TR<T, 6, TH, CX>(a);
        case 7: return launch_fused_TR<T, 7, TH, CX>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TH, int CX>
hipError_t launch_fused(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_fused_T<F32, TH, CX>(a);
        case ICL_F16: return launch_fused_T<F16, TH, CX>(a);
        default: return launch_fused_T<BF16, TH, CX>(a);
    }
}

bool supports_fused(const SepArgs& a) { return a.r >= 0 && a.r <= 7; }

// Persistent fused variant: each block walks tiles with stride gridDim.x and keeps the
// next tile's global loads in flight (registers) while the current tile's row and
// column passes run from LDS.  Two barriers per tile.
template <class T, int R, int TH, int CX>
__global__ __launch_bounds__(256) void sep_pers(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                size_t dp, int W, int H, const float* __restrict__ tx,
                                                const float* __restrict__ ty, int tiles_x, int tiles_y, int vec_ok,
                                                int vec_out, Border bd) {
    using G = SepTile<R, TH, CX>;
    constexpr int TW = G::TW, RA = G::RA, LW = G::LW, NR = G::NR;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    float* in_s = lds;
    float* t_s = lds + NR * LW;
    Stage<T, NR, LW> st;
    const BandWalk walk(tiles_x, tiles_y);
    int t = walk.tile(0);
    if (t < 0) return;
    int x0, y0;
    tile_origin(t, tiles_x, TW, TH, x0, y0);
    st.load(src, sp, W, H, x0 - RA, y0 - R, vec_ok, bd);
    st.store(in_s);
    __syncthreads();
    // Pipeline per tile: issue the next tile's loads, run the row pass, then (after the
    // barrier that frees in_s) move the prefetched registers into in_s BEFORE this tile's
    // output stores are issued, so the wait on the loads never waits on stores too.
    for (int k = 0; t >= 0; ++k) {
        const int tn = walk.tile(k + 1);
        if (tn >= 0) {
            int nx0, ny0;
            tile_origin(tn, tiles_x, TW, TH, nx0, ny0);
            st.load(src, sp, W, H, nx0 - RA, ny0 - R, vec_ok, bd);
        }
        sep_row_pass<R, TH, CX>(in_s, t_s, tx);
        __syncthreads();
        if (tn >= 0) st.store(in_s);
        sep_col_pass<T, R, TH, CX>(t_s, dst, dp, W, H, ty, x0, y0, vec_out);
        __syncthreads();
        t = tn;
        if (t >= 0) tile_origin(t, tiles_x, TW, TH, x0, y0);
    }
}

template <class T, int R, int TH, int CX>
hipError_t launch_pers_TR(const SepArgs& a) {
    using G = SepTile<R, TH, CX>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + TH - 1) / TH;
    const size_t al = 4 * (size_t)T::size;
    const int vec_ok = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0);
    const int vec_out = ((uintptr_t)a.dst % al == 0) && (a.dp % al == 0);
    const void* k = reinterpret_cast<const void*>(&sep_pers<T, R, TH, CX>);
    hipLaunchKernelGGL((sep_pers<T, R, TH, CX>), dim3(persistent_grid(k, 256, tiles_x * tiles_y)), dim3(256), 0,
                       a.st, a.src, a.sp, a.dst, a.dp, a.W, a.H, a.tx, a.ty, tiles_x, tiles_y, vec_ok, vec_out,
                       a.bd);
    return hipGetLastError();
}

template <class T, int TH, int CX>
hipError_t launch_pers_T(const SepArgs& a) {
    switch (a.r) {
        case 0: return launch_pers_TR<T, 0, TH, CX>(a);
        case 1: return launch_pers_TR<T, 1, TH, CX>(a);
        case 2: return launch_pers_TR<T, 2, TH, CX>(a);
        case 3: return launch_pers_TR<T, 3, TH, CX>(a);
        case 4: return launch_pers_TR<T, 4, TH, CX>(a);
        case 5: return launch_pers_TR<T, 5, TH, CX>(a);
        case 6: return launch_pers_TR<T, 6, TH, CX>(a);
        case 7: return launch_pers_TR<T, 7, TH, CX>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TH, int CX>
hipError_t launch_pers(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_pers_T<F32, TH, CX>(a);
        case ICL_F16: return launch_pers_T<F16, TH, CX>(a);
        default: return launch_pers_T<BF16, TH, CX>(a);
    }
}

// ------------------------------------------------------------------ image-memory stand-in
// The paper's image-memory candidate reads pixels through the texture unit, whose sampler
// applies the boundary condition (Section 5.2).  gfx950 has no image instructions; the
// nearest it has is a buffer descriptor, whose hardware range check returns 0 for any read
// at or past the descriptor's size.  Here each staged row is read through a descriptor of
// its own, wave-uniform: base at the row, size W pixels for a row inside the image and 0
// for a row outside.  With the constant boundary at 0 the hardware then supplies both
// bounds: a column left of the image is a negative (as unsigned, huge) offset and a column
// at or right of W an offset past the size, so the staging has no boundary arithmetic at
// all.  With the clamp boundary the offsets are clamped (the row by its base, the column in
// software, as the sampler's clamp-to-edge mode would); a nonzero constant is applied after
// the read.  One pixel per lane and load (a dword or short buffer load), each wave a row.
template <class T> __device__ __forceinline__ float decode1(unsigned bits);
template <> __device__ __forceinline__ float decode1<F32>(unsigned b) { return __uint_as_float(b); }
template <> __device__ __forceinline__ float decode1<F16>(unsigned b) {
    return decode(__builtin_bit_cast(_Float16, (unsigned short)b));
}
template <> __device__ __forceinline__ float decode1<BF16>(unsigned b) { return __uint_as_float(b << 16); }

template <class T, int NR, int LW>
__device__ __forceinline__ void stage_rows_img(const void* __restrict__ src, size_t sp, int W, int H, int gx0, int gy0,
                                               Border bd, float* __restrict__ in_s) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    const bool cst = bd.constant != 0, cnz = cst && bd.value != 0.f;
    for (int rr = wave; rr < NR; rr += 4) {
        const int y = gy0 + rr;
        const bool yin = y >= 0 && y < H;
        const char* base = static_cast<const char*>(src) + (size_t)clampi(y, H) * sp;
        const Rsrc rs = make_rsrc(base, (cst && !yin) ? 0u : (unsigned)W * T::size);
#pragma unroll
        for (int c0 = 0; c0 < LW; c0 += 64) {
            const int c = c0 + lane;
            if (LW % 64 != 0 && c >= LW) break;
            const int x = gx0 + c;
            const unsigned off = (unsigned)(cst ? x : clampi(x, W)) * (unsigned)T::size;
            float v = decode1<T>(bload1_raw<T>(rs, off));
            if (cnz && (!yin || x < 0 || x >= W)) v = bd.value;
            in_s[rr * LW + c] = v;
        }
    }
}

// The same with four pixels per lane: a row's LW/4 chunks start at a multiple of 4 columns
// (x0 - RA), so a chunk left of the image is wholly left of it, and the range check, which
// this hardware applies to each dword of a wider load (a 16-byte load that crosses the
// descriptor's end returns its in-range dwords and zeros), zeroes the part of a chunk past
// W.  So for float32 (and half types with an even width, where no dword holds a pixel on
// each side of W) the constant-0 boundary still costs no boundary arithmetic.  Clamp: a chunk
// not wholly inside reads its pixels one by one through the clamp.
// vec false (rows not 4-pixel aligned, or a half type with an odd width): every chunk is
// read pixel by pixel through the same row descriptor.
template <class T, int NR, int LW>
__device__ __forceinline__ void stage_rows_img4(const void* __restrict__ src, size_t sp, int W, int H, int gx0,
                                                int gy0, Border bd, float* __restrict__ in_s, bool vec) {
    constexpr int C4 = LW / 4;
    static_assert(C4 <= 64, "one chunk per lane");
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    const bool cst = bd.constant != 0, cnz = cst && bd.value != 0.f;
    if (lane >= C4) return;   // lanes past the row's chunks have nothing to stage
    for (int rr = wave; rr < NR; rr += 4) {
        const int y = gy0 + rr;
        const bool yin = y >= 0 && y < H;
        const char* base = static_cast<const char*>(src) + (size_t)clampi(y, H) * sp;
        const Rsrc rs = make_rsrc(base, (cst && !yin) ? 0u : (unsigned)W * T::size);
        const int x = gx0 + 4 * lane;
        v4f v;
        if (vec && (cst || (x >= 0 && x + 4 <= W))) {
            v = decode4<T>(bload4_raw<T>(rs, (unsigned)x * T::size));
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = decode1<T>(bload1_raw<T>(rs, (unsigned)(cst ? x + q : clampi(x + q, W)) * T::size));
        }
        if (cnz) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (!yin || x + q < 0 || x + q >= W) v[q] = bd.value;
        }
        lds4(&in_s[rr * LW + 4 * lane], v);
    }
}

template <class T, int R, int TH, int CX, bool X4>
__global__ __launch_bounds__(256) void sep_fused_img(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                     size_t dp, int W, int H, const float* __restrict__ tx,
                                                     const float* __restrict__ ty, int tiles_x, int vec_in, int vec_out,
                                                     Border bd) {
    using G = SepTile<R, TH, CX>;
    __shared__ __attribute__((aligned(16))) float lds[G::LDS_FLOATS];
    float* in_s = lds;
    float* t_s = lds + G::NR * G::LW;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (int)(t % (unsigned)tiles_x) * G::TW;
    const int y0 = (int)(t / (unsigned)tiles_x) * TH;
    if constexpr (X4) stage_rows_img4<T, G::NR, G::LW>(src, sp, W, H, x0 - G::RA, y0 - R, bd, in_s, vec_in != 0);
    else stage_rows_img<T, G::NR, G::LW>(src, sp, W, H, x0 - G::RA, y0 - R, bd, in_s);
    __syncthreads();
    sep_row_pass<R, TH, CX>(in_s, t_s, tx);
    __syncthreads();
    sep_col_pass<T, R, TH, CX>(t_s, dst, dp, W, H, ty, x0, y0, vec_out != 0);
}

template <class T, int R, int TH, int CX, bool X4>
hipError_t launch_img_TR(const SepArgs& a) {
    using G = SepTile<R, TH, CX>;
    const int tiles_x = (a.W + G::TW - 1) / G::TW;
    const int tiles_y = (a.H + TH - 1) / TH;
    const size_t al = 4 * (size_t)T::size;
    const int vec_out = ((uintptr_t)a.dst % al == 0) && (a.dp % al == 0);
    const int vec_in = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0) && (T::size == 4 || a.W % 2 == 0);
    hipLaunchKernelGGL((sep_fused_img<T, R, TH, CX, X4>), dim3(tiles_x * tiles_y), dim3(256), 0, a.st, a.src, a.sp,
                       a.dst, a.dp, a.W, a.H, a.tx, a.ty, tiles_x, vec_in, vec_out, a.bd);
    return hipGetLastError();
}

template <class T, int TH, int CX, bool X4>
hipError_t launch_img_T(const SepArgs& a) {
    switch (a.r) {
        case 0: return launch_img_TR<T, 0, TH, CX, X4>(a);
        case 1: return launch_img_TR<T, 1, TH, CX, X4>(a);
        case 2: return launch_img_TR<T, 2, TH, CX, X4>(a);
        case 3: return launch_img_TR<T, 3, TH, CX, X4>(a);
        case 4: return launch_img_TR<T, 4, TH, CX, X4>(a);
        case 5: return launch_img_TR<T, 5, TH, CX, X4>(a);
        case 6: return launch_img_TR<T, 6, TH, CX, X4>(a);
        case 7: return launch_img_TR<T, 7, TH, CX, X4>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TH, int CX, bool X4>
hipError_t launch_img(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_img_T<F32, TH, CX, X4>(a);
        case ICL_F16: return launch_img_T<F16, TH, CX, X4>(a);
        default: return launch_img_T<BF16, TH, CX, X4>(a);
    }
}

// the row descriptors address a row with 32-bit offsets: the row must be under 2^31 bytes
bool supports_img(const SepArgs& a) {
    return supports_fused(a) && (size_t)a.W * (a.dt == ICL_F32 ? 4 : 2) < ((size_t)1 << 31);
}


// ------------------------------------------------------------------ column walk
// Persistent work-groups take items (64-column strip, segment of SEG rows) in row-major
// order of segments (the items running side by side are horizontal neighbours, sharing
// their halo columns in L2) and walk each down in 64-row steps (sep_colwalk.hpp): every
// input row of a segment is staged and row-passed once.
template <class T, int R, int SEG>
__global__ __launch_bounds__(256, 4) void sep_colwalk(DevImage d, int nstrips, int nitems, Border bd) {
    using G = ColGeom<1, 64>;
    __shared__ __attribute__((aligned(16))) float in_s[G::IN_FLOATS];
    __shared__ __attribute__((aligned(16))) float t_s[G::T_FLOATS];
    for (int i = first_tile(); i < nitems; i += (int)gridDim.x) {
        const int seg = i / nstrips, strip = i - seg * nstrips;
        const ColItem it{0, strip * 64, seg * SEG, min(SEG, d.H - seg * SEG)};
        col_item<T, R>(d, it, in_s, t_s, bd);
    }
}

template <class T, int R, int SEG>
hipError_t launch_colwalk_TR(const SepArgs& a) {
    const size_t al = 4 * (size_t)T::size;
    DevImage d{};
    d.src = a.src; d.dst = a.dst; d.sp = a.sp; d.dp = a.dp; d.tx = a.tx; d.ty = a.ty;
    d.W = a.W; d.H = a.H; d.r = R;
    d.vec_ok = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0);
    d.vec_out = ((uintptr_t)a.dst % al == 0) && (a.dp % al == 0);
    d.src_bytes = (unsigned)((size_t)(a.H - 1) * a.sp + (size_t)a.W * T::size);
    const int nstrips = (a.W + 63) / 64, nsegs = (a.H + SEG - 1) / SEG;
    const void* k = reinterpret_cast<const void*>(&sep_colwalk<T, R, SEG>);
    hipLaunchKernelGGL((sep_colwalk<T, R, SEG>), dim3(persistent_grid(k, 256, nstrips * nsegs)), dim3(256), 0, a.st, d,
                       nstrips, nstrips * nsegs, a.bd);
    return hipGetLastError();
}

template <class T, int SEG>
hipError_t launch_colwalk_T(const SepArgs& a) {
    switch (a.r) {
        case 0: return launch_colwalk_TR<T, 0, SEG>(a);
        case 1: return launch_colwalk_TR<T, 1, SEG>(a);
        case 2: return launch_colwalk_TR<T, 2, SEG>(a);
        case 3: return launch_colwalk_TR<T, 3, SEG>(a);
        case 4: return launch_colwalk_TR<T, 4, SEG>(a);
        case 5: return launch_colwalk_TR<T, 5, SEG>(a);
        case 6: return launch_colwalk_TR<T, 6, SEG>(a);
        case 7: return launch_colwalk_TR<T, 7, SEG>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int SEG>
hipError_t launch_colwalk(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_colwalk_T<F32, SEG>(a);
        case ICL_F16: return launch_colwalk_T<F16, SEG>(a);
        default: return launch_colwalk_T<BF16, SEG>(a);
    }
}

// the source extent and pitch must fit 31-bit buffer offsets
bool supports_colwalk(const SepArgs& a) {
    const size_t es = a.dt == ICL_F32 ? 4 : 2;
    return supports_fused(a) && a.sp < ((size_t)1 << 31) &&
           (size_t)(a.H - 1) * a.sp + (size_t)a.W * es < ((size_t)1 << 31) &&
           (long long)((a.W + 63) / 64) * ((a.H + 63) / 64) < 0x7fffffffLL;
}

// ------------------------------------------------------------------ register strips
template <class T, int R, int TH>
__global__ __launch_bounds__(64) void sep_strip(const void* __restrict__ src, size_t sp, void* __restrict__ dst,
                                                size_t dp, int W, int H, const float* __restrict__ tx,
                                                const float* __restrict__ ty, int nstrips, int vec_in, int vec_out,
                                                Border bd) {
    const int strip = (int)(blockIdx.x % (unsigned)nstrips);
    const int y0 = (int)(blockIdx.x / (unsigned)nstrips) * TH;
    sep_strip_body<T, R, TH>(src, sp, dst, dp, W, H, tx, ty, strip * StripGeom<R>::SW, y0, vec_in != 0,
                             vec_out != 0, bd);
}

template <class T, int R, int TH>
hipError_t launch_strip_TR(const SepArgs& a) {
    const int nstrips = (a.W + StripGeom<R>::SW - 1) / StripGeom<R>::SW;
    const int rows = (a.H + TH - 1) / TH;
    const size_t al = 4 * (size_t)T::size;
    const int vec_in = ((uintptr_t)a.src % al == 0) && (a.sp % al == 0);
    const int vec_out = ((uintptr_t)a.dst % al == 0) && (a.dp % al == 0);
    hipLaunchKernelGGL((sep_strip<T, R, TH>), dim3((unsigned)(nstrips * rows)), dim3(64), 0, a.st, a.src, a.sp, a.dst,
                       a.dp, a.W, a.H, a.tx, a.ty, nstrips, vec_in, vec_out, a.bd);
    return hipGetLastError();
}

template <class T, int TH>
hipError_t launch_strip_T(const SepArgs& a) {
    switch (a.r) {
        case 0: return launch_strip_TR<T, 0, TH>(a);
        case 1: return launch_strip_TR<T, 1, TH>(a);
        case 2: return launch_strip_TR<T, 2, TH>(a);
        case 3: return launch_strip_TR<T, 3, TH>(a);
        case 4: return launch_strip_TR<T, 4, TH>(a);
        case 5: return launch_strip_TR<T, 5, TH>(a);
        case 6: return launch_strip_TR<T, 6, TH>(a);
        case 7: return launch_strip_TR<T, 7, TH>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int TH>
hipError_t launch_strip(const SepArgs& a) {
    switch (a.dt) {
        case ICL_F32: return launch_strip_T<F32, TH>(a);
        case ICL_F16: return launch_strip_T<F16, TH>(a);
        default: return launch_strip_T<BF16, TH>(a);
    }
}

const Variant<SepArgs> kSep[] = {
    {"plain2p", supports_plain, launch_plain},
    {"fused_t32_c1", supports_fused, launch_fused<32, 1>},
    {"fused_t64_c1", supports_fused, launch_fused<64, 1>},
    {"fused_t32_c2", supports_fused, launch_fused<32, 2>},
    {"fused_t16_c2", supports_fused, launch_fused<16, 2>},
    {"pers_t32_c1", supports_fused, launch_pers<32, 1>},
    {"pers_t16_c2", supports_fused, launch_pers<16, 2>},
    {"pers_t64_c1", supports_fused, launch_pers<64, 1>},
    {"pers_t16_c1", supports_fused, launch_pers<16, 1>},
    {"strip_t32", supports_fused, launch_strip<32>},
    {"strip_t16", supports_fused, launch_strip<16>},
    {"strip_t64", supports_fused, launch_strip<64>},
    {"fused_img_t32_c1", supports_img, launch_img<32, 1, false>},
    {"fused_img_t16_c2", supports_img, launch_img<16, 2, false>},
    {"fused_img4_t32_c1", supports_img, launch_img<32, 1, true>},
    {"fused_img4_t16_c2", supports_img, launch_img<16, 2, true>},
    {"colwalk_s64", supports_colwalk, launch_colwalk<64>},
    {"colwalk_s128", supports_colwalk, launch_colwalk<128>},
    {"colwalk_s256", supports_colwalk, launch_colwalk<256>},
};

}  // namespace

size_t sep_workspace(int W, int H) { return (size_t)W * (size_t)H * sizeof(float); }

const Variant<SepArgs>* sep_variants(int* count) {
    *count = (int)(sizeof(kSep) / sizeof(kSep[0]));
    return kSep;
}

int sep_default(const SepArgs& a) { return supports_fused(a) ? 1 : 0; }

}  // namespace icl
