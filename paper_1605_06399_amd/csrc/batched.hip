// Batched separable convolution over images of uneven size and radius in one
// persistent launch.  The host turns the batch into a table of 64x64 output
// tiles, each naming its image; a grid sized to the device's resident capacity
// walks the table with a fixed stride, and each tile runs the same fused
// single-pass body as icl_conv_sep (row pass into LDS, column pass from LDS),
// instantiated per radius and picked by a wave-uniform branch on the image's
// radius.  Launch arguments are only the two tables, so the launch captures into
// a HIP graph as one kernel node and replays re-read images and taps.
//
// Variants
//   persistent_fused_t64 : the tile walk above (64x64 output tiles, LDS passes).
//   persistent_fused_t64_rsort, persistent_fused_t32_rsort : the same walk over 64- or
//                          32-row tiles ordered by decreasing radius.
//   persistent_strip_t32 : a persistent grid of single waves walking a table of
//                          (image, strip, 32-row block) items with the register-
//                          streaming body of the per-image strip variant; the items
//                          are sorted by radius, so the waves resident at a time mostly
//                          run the same radius body.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "sep_strip.hpp"
#include "sep_colwalk.hpp"
#include "sep_tile.hpp"
#include "tile_stage.hpp"

namespace icl {

struct BatchTile {
    int img, x0, y0, r;   // r: the image's radius (orders the tiles on the host)
};

struct StripItem {
    int img, xs, y0, r;
};

namespace {

constexpr int BCX = 1;     // tile columns = 64 * BCX
constexpr int RMAX = 7;

// Persistent walk over the tile table.  The next tile's descriptor and pixels are
// fetched into registers while the current tile is computed; the row-pass
// intermediate lives at a fixed LDS offset past the largest staged tile, so staging
// the next tile (any radius) never overlaps a column pass still reading.
template <class T, int BTH>
__global__ __launch_bounds__(256) void sep_batched_k(const DevImage* __restrict__ imgs,
                                                     const BatchTile* __restrict__ tiles, int ntiles) {
    constexpr int TW = 64 * BCX;
    constexpr int IN_MAX = SepTile<RMAX, BTH, BCX>::NR * SepTile<RMAX, BTH, BCX>::LW;
    __shared__ __attribute__((aligned(16))) float lds[SepTile<RMAX, BTH, BCX>::LDS_FLOATS];
    float* in_s = lds;
    float* t_s = lds + IN_MAX;
    RStage<T, BTH + 2 * RMAX> rs;
    int t = first_tile();
    if (t >= ntiles) return;
    BatchTile bt = tiles[t];
    DevImage d = imgs[bt.img];
    auto fetch = [&](const DevImage& im, const BatchTile& b) {
        const int ra = (im.r + 3) & ~3;
        rs.load(im.src, im.sp, im.W, im.H, b.x0 - ra, b.y0 - im.r, BTH + 2 * im.r, (TW + 2 * ra) / 4, im.vec_ok);
    };
    fetch(d, bt);
    rs.store(in_s, BTH + 2 * d.r, (TW + 2 * ((d.r + 3) & ~3)) / 4);
    __syncthreads();
    // Per tile: issue the next tile's loads, row pass, barrier, move the prefetched
    // registers into in_s before this tile's output stores are issued, column pass, barrier.
    for (;;) {
        const int tn = t + (int)gridDim.x;
        BatchTile nbt = bt;
        DevImage nd = d;
        if (tn < ntiles) {
            nbt = tiles[tn];
            nd = imgs[nbt.img];
            fetch(nd, nbt);
        }
        switch (d.r) {
#define ICL_BATCH_CASE(R)                                                                        \
    case R:                                                                                      \
        sep_row_pass<R, BTH, BCX>(in_s, t_s, d.tx);                                              \
        __syncthreads();                                                                         \
        if (tn < ntiles) rs.store(in_s, BTH + 2 * nd.r, (TW + 2 * ((nd.r + 3) & ~3)) / 4);       \
        sep_col_pass<T, R, BTH, BCX>(t_s, d.dst, d.dp, d.W, d.H, d.ty, bt.x0, bt.y0, d.vec_out); \
        break;
            ICL_BATCH_CASE(0)
            ICL_BATCH_CASE(1)
            ICL_BATCH_CASE(2)
            ICL_BATCH_CASE(3)
            ICL_BATCH_CASE(4)
            ICL_BATCH_CASE(5)
            ICL_BATCH_CASE(6)
            ICL_BATCH_CASE(7)
#undef ICL_BATCH_CASE
            default: break;
        }
        __syncthreads();
        if (tn >= ntiles) break;
        t = tn;
        bt = nbt;
        d = nd;
    }
}

constexpr int STH = 32;   // rows per strip item

// Persistent strip walk: wave i takes items i, i + grid, ...
template <class T>
__global__ __launch_bounds__(64) void sep_batched_strip_k(const DevImage* __restrict__ imgs,
                                                          const StripItem* __restrict__ items, int nitems) {
    for (int i = (int)blockIdx.x; i < nitems; i += (int)gridDim.x) {
        const StripItem it = items[i];
        const DevImage d = imgs[it.img];
        switch (it.r) {
#define ICL_STRIP_CASE(R)                                                                                   \
    case R:                                                                                                 \
        sep_strip_body<T, R, STH>(d.src, d.sp, d.dst, d.dp, d.W, d.H, d.tx, d.ty, it.xs, it.y0, d.vec_ok != 0, \
                                  d.vec_out != 0);                                                          \
        break;
            ICL_STRIP_CASE(0)
            ICL_STRIP_CASE(1)
            ICL_STRIP_CASE(2)
            ICL_STRIP_CASE(3)
            ICL_STRIP_CASE(4)
            ICL_STRIP_CASE(5)
            ICL_STRIP_CASE(6)
            ICL_STRIP_CASE(7)
#undef ICL_STRIP_CASE
            default: break;
        }
    }
}

// Items are ordered by decreasing radius; end[R] is one past the last item of radius R (the
// radius-7 items come first).  A work-group takes items b, b + grid, b + 2 grid, ... of that
// order, and the walk is split into one loop per radius, so each loop's body is compiled for
// its radius alone (one loop with a switch over the radius would hold the registers of all
// eight bodies at once).
struct ColRanges {
    int end[RMAX + 1];
};

// The register budget is set for the work-groups the LDS admits: four per CU for 64-column
// strips with 64-row steps (40 KB), three for 128-column strips with 32-row steps (42 KB).
template <class T, int CX, int STEP>
__global__ __launch_bounds__(256, CX == 1 ? 4 : 3) void sep_batched_col_k(const DevImage* __restrict__ imgs,
                                                                         const ColItem* __restrict__ items,
                                                                         ColRanges rg) {
    using G = ColGeom<CX, STEP>;
    __shared__ __attribute__((aligned(16))) float in_s[G::IN_FLOATS];
    __shared__ __attribute__((aligned(16))) float t_s[G::T_FLOATS];
    int i = first_tile();
    static_for<RMAX + 1>([&](auto k) {
        constexpr int R = RMAX - decltype(k)::value;
        for (; i < rg.end[R]; i += (int)gridDim.x) {
            const ColItem li = items[i];
            const ColItem it{uni(li.img), uni(li.x0), uni(li.y0), uni(li.rows)};
            const DevImage d = uni(imgs[it.img]);
            col_item<T, R, CX, STEP>(d, it, in_s, t_s);
        }
    });
}

}  // namespace

// the tile walk: on the 256-image workload the strip walk's waves hold too many registers
// (two waves per SIMD) and it runs at about half the tile walk's rate
int batched_default() { return 0; }

namespace {

int strip_width(int r) {
    switch (r) {
        case 0: return StripGeom<0>::SW;
        case 1: case 2: case 3: case 4: return StripGeom<4>::SW;
        default: return StripGeom<7>::SW;
    }
}

}  // namespace
}  // namespace icl

using namespace icl;

// Tile tables of the tile-walk variants: 64-row tiles in image order, 64-row tiles with
// the largest radius first, 32-row tiles with the largest radius first.
constexpr int NWALKS = 3;
// Column walks: 64-column strips in 64-row steps over segments of 256, 512, 2048 (a whole
// image of the usual batch), 128 and 64 rows; 128-column strips in 32-row steps over segments
// of 128 and 256 rows.
constexpr int NCOL = 7;
constexpr int kColSeg[NCOL] = {256, 512, 2048, 128, 64, 128, 256};
constexpr int kColCx[NCOL] = {1, 1, 1, 1, 1, 2, 2};
constexpr int kFirstCol = 4;   // variant index of the first column walk

struct icl_batch_plan {
    icl_dtype dt;
    DevImage* d_imgs;
    BatchTile* d_tiles[NWALKS];
    int ntiles[NWALKS];
    int grid[NWALKS];
    StripItem* d_items;
    int nitems;
    int strip_grid;
    ColItem* d_col[NCOL];
    int ncol[NCOL];
    ColRanges col_rg[NCOL];
    int col_grid[NCOL];
    bool col_ok;   // every image's source extent fits a 31-bit buffer offset
    long long pixels;
    int nimg, rmax;
    int tuned;   // walk picked by icl_batch_plan_tune, -1 before
};

namespace {

constexpr int walk_rows(int w) { return w == 2 ? 32 : 64; }

template <class T>
const void* batched_kernel(int walk) {
    return walk == 2 ? reinterpret_cast<const void*>(&sep_batched_k<T, 32>)
                     : reinterpret_cast<const void*>(&sep_batched_k<T, 64>);
}

const void* kernel_for(icl_dtype dt, int walk) {
    switch (dt) {
        case ICL_F32: return batched_kernel<F32>(walk);
        case ICL_F16: return batched_kernel<F16>(walk);
        default: return batched_kernel<BF16>(walk);
    }
}

template <class T>
void launch_walk(const icl_batch_plan* p, int w, hipStream_t st) {
    if (w == 2)
        hipLaunchKernelGGL((sep_batched_k<T, 32>), dim3(p->grid[w]), dim3(256), 0, st, p->d_imgs, p->d_tiles[w],
                           p->ntiles[w]);
    else
        hipLaunchKernelGGL((sep_batched_k<T, 64>), dim3(p->grid[w]), dim3(256), 0, st, p->d_imgs, p->d_tiles[w],
                           p->ntiles[w]);
}

template <int CX, int STEP>
const void* col_kernel_cx(icl_dtype dt) {
    switch (dt) {
        case ICL_F32: return reinterpret_cast<const void*>(&sep_batched_col_k<F32, CX, STEP>);
        case ICL_F16: return reinterpret_cast<const void*>(&sep_batched_col_k<F16, CX, STEP>);
        default: return reinterpret_cast<const void*>(&sep_batched_col_k<BF16, CX, STEP>);
    }
}
const void* col_kernel_for(icl_dtype dt, int cx) { return cx == 1 ? col_kernel_cx<1, 64>(dt) : col_kernel_cx<2, 32>(dt); }

const void* strip_kernel_for(icl_dtype dt) {
    switch (dt) {
        case ICL_F32: return reinterpret_cast<const void*>(&sep_batched_strip_k<F32>);
        case ICL_F16: return reinterpret_cast<const void*>(&sep_batched_strip_k<F16>);
        default: return reinterpret_cast<const void*>(&sep_batched_strip_k<BF16>);
    }
}

bool ranges_overlap(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) { return a0 < b1 && b0 < a1; }

// The plan's problem class for the tune cache: storage type, largest radius, tile count
// (size class) and image count.
Problem plan_problem(const icl_batch_plan* p) {
    return Problem{ICL_OP_CONV_SEP_BATCHED, p->dt, p->rmax, std::max(p->ntiles[0], 1), 64 * 64, 1, 1,
                   std::max(p->nimg, 1)};
}

// the first column walk where it can address every image, else the tile walk
int plan_default(const icl_batch_plan* p) { return p->col_ok ? kFirstCol : batched_default(); }

int plan_variant(const icl_batch_plan* p) {
    int v = (variant_forced(ICL_OP_CONV_SEP_BATCHED) || p->tuned < 0) ? select_variant(plan_problem(p), plan_default(p))
                                                                      : p->tuned;
    // a cached column walk for a plan whose images it cannot address takes the default
    if (v >= kFirstCol && !p->col_ok && !variant_forced(ICL_OP_CONV_SEP_BATCHED)) v = plan_default(p);
    return v;
}

// Order-independent digest of every output pixel of a plan (sum over pixels of a SplitMix64
// mix of image, position and stored bits, modulo 2^64), for the tuner's bit-exact check.
template <class T>
__global__ __launch_bounds__(256) void batch_digest_k(const DevImage* __restrict__ imgs,
                                                      const BatchTile* __restrict__ tiles, int ntiles,
                                                      unsigned long long* out) {
    unsigned long long h = 0;
    for (int t = (int)blockIdx.x; t < ntiles; t += (int)gridDim.x) {
        const BatchTile bt = tiles[t];
        const DevImage d = imgs[bt.img];
        for (int q = (int)threadIdx.x; q < 64 * 64; q += 256) {
            const int x = bt.x0 + (q & 63), y = bt.y0 + (q >> 6);
            if (x >= d.W || y >= d.H) continue;
            const unsigned char* p = static_cast<const unsigned char*>(d.dst) + (size_t)y * d.dp + (size_t)x * T::size;
            unsigned long long bits = T::size == 4 ? *reinterpret_cast<const unsigned*>(p)
                                                   : *reinterpret_cast<const unsigned short*>(p);
            unsigned long long z = bits + ((unsigned long long)bt.img << 40) + ((unsigned long long)y << 20) +
                                   (unsigned long long)x + 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            h += z ^ (z >> 31);
        }
    }
    atomicAdd(out, h);
}

hipError_t plan_digest(const icl_batch_plan* p, unsigned long long* d_out, unsigned long long* h_out, hipStream_t st) {
    hipError_t e = hipMemsetAsync(d_out, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    const int grid = std::min(std::max(p->ntiles[0], 1), 4096);
    switch (p->dt) {
        case ICL_F32: hipLaunchKernelGGL(batch_digest_k<F32>, dim3(grid), dim3(256), 0, st, p->d_imgs, p->d_tiles[0],
                                         p->ntiles[0], d_out); break;
        case ICL_F16: hipLaunchKernelGGL(batch_digest_k<F16>, dim3(grid), dim3(256), 0, st, p->d_imgs, p->d_tiles[0],
                                         p->ntiles[0], d_out); break;
        default: hipLaunchKernelGGL(batch_digest_k<BF16>, dim3(grid), dim3(256), 0, st, p->d_imgs, p->d_tiles[0],
                                    p->ntiles[0], d_out); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h_out, d_out, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

hipError_t launch_plan(const icl_batch_plan* plan, int v, hipStream_t st);

}  // namespace

extern "C" {

icl_status icl_batch_plan_create(const icl_image_desc* descs, int count, icl_dtype dtype, icl_batch_plan** plan) {
    if (!plan) return ICL_ERR_INVALID_VALUE;
    *plan = nullptr;
    if (count < 0 || (count > 0 && !descs)) return ICL_ERR_INVALID_VALUE;
    if (dtype != ICL_F32 && dtype != ICL_F16 && dtype != ICL_BF16) return ICL_ERR_DTYPE;
    const int es = elem_size(dtype);
    std::vector<DevImage> imgs;
    std::vector<BatchTile> tiles[NWALKS];
    std::vector<StripItem> items;
    long long pixels = 0;
    const size_t al = 4 * (size_t)es;
    for (int i = 0; i < count; ++i) {
        const icl_image_desc& d = descs[i];
        if (d.width < 0 || d.height < 0) return ICL_ERR_INVALID_VALUE;
        if (d.radius < 0 || d.radius > RMAX) return ICL_ERR_RADIUS;
        if (d.width == 0 || d.height == 0) {
            imgs.push_back(DevImage{});
            continue;
        }
        if (!d.src || !d.dst || !d.taps_x || !d.taps_y) return ICL_ERR_INVALID_VALUE;
        if (d.src_pitch < (size_t)d.width * es || d.src_pitch % es || d.dst_pitch < (size_t)d.width * es ||
            d.dst_pitch % es)
            return ICL_ERR_PITCH;
        const uintptr_t s0 = (uintptr_t)d.src, s1 = s0 + (size_t)(d.height - 1) * d.src_pitch + (size_t)d.width * es;
        const uintptr_t o0 = (uintptr_t)d.dst, o1 = o0 + (size_t)(d.height - 1) * d.dst_pitch + (size_t)d.width * es;
        if (ranges_overlap(s0, s1, o0, o1)) return ICL_ERR_ALIAS;
        DevImage di;
        di.src = d.src; di.dst = d.dst; di.sp = d.src_pitch; di.dp = d.dst_pitch;
        di.tx = d.taps_x; di.ty = d.taps_y; di.W = d.width; di.H = d.height; di.r = d.radius;
        di.vec_ok = ((uintptr_t)d.src % al == 0) && (d.src_pitch % al == 0);
        di.vec_out = ((uintptr_t)d.dst % al == 0) && (d.dst_pitch % al == 0);
        const size_t ext = (size_t)(d.height - 1) * d.src_pitch + (size_t)d.width * es;
        di.src_bytes = ext < ((size_t)1 << 31) ? (unsigned)ext : 0u;
        imgs.push_back(di);
        pixels += (long long)d.width * d.height;
        const int tx = (d.width + 64 * BCX - 1) / (64 * BCX);
        for (int w = 0; w < NWALKS; w += 1) {
            if (w == 1) continue;   // the sorted copy of walk 0 is made below
            const int th = walk_rows(w), ty = (d.height + th - 1) / th;
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) tiles[w].push_back(BatchTile{i, x * 64 * BCX, y * th, d.radius});
        }
        const int sw = strip_width(d.radius);
        const int sx = (d.width + sw - 1) / sw, sy = (d.height + STH - 1) / STH;
        for (int y = 0; y < sy; ++y)
            for (int x = 0; x < sx; ++x) items.push_back(StripItem{i, x * sw, y * STH, d.radius});
    }
    // largest radius first (the longest work first, and the resident waves mostly run one
    // radius body at a time), then image, row, column
    std::stable_sort(items.begin(), items.end(),
                     [](const StripItem& a, const StripItem& b) { return a.r > b.r; });
    // column-walk items: images by decreasing radius, then by decreasing work of one item
    // (segment rows x (2r + 3)), so the longest items start first; inside an image by
    // segment, then column, so the items running side by side share their halo columns
    std::vector<ColItem> cols[NCOL];
    bool col_ok = true;
    {
        std::vector<int> order;
        for (int i = 0; i < (int)imgs.size(); ++i)
            if (imgs[i].src) order.push_back(i);
        for (int c = 0; c < NCOL; ++c) {
            const int seg = kColSeg[c];
            auto work = [&](int i) { return (long long)std::min(imgs[i].H, seg) * (2 * imgs[i].r + 3); };
            std::vector<int> o = order;
            std::stable_sort(o.begin(), o.end(), [&](int a, int b) {
                return imgs[a].r != imgs[b].r ? imgs[a].r > imgs[b].r : work(a) > work(b);
            });
            const int cw = 64 * kColCx[c];
            for (int i : o) {
                const DevImage& d = imgs[i];
                for (int y = 0; y < d.H; y += seg)
                    for (int x = 0; x < d.W; x += cw) cols[c].push_back(ColItem{i, x, y, std::min(seg, d.H - y)});
            }
        }
        for (const DevImage& d : imgs)
            if (d.src && (d.src_bytes == 0 || d.sp >= ((size_t)1 << 31))) col_ok = false;
    }
    tiles[1] = tiles[0];
    auto by_radius = [](const BatchTile& a, const BatchTile& b) { return a.r > b.r; };
    std::stable_sort(tiles[1].begin(), tiles[1].end(), by_radius);
    std::stable_sort(tiles[2].begin(), tiles[2].end(), by_radius);
    // outputs of different images must not overlap each other or any input
    {
        std::vector<std::pair<uintptr_t, uintptr_t>> outs, ins;
        for (const DevImage& d : imgs) {
            if (!d.src) continue;
            outs.push_back({(uintptr_t)d.dst, (uintptr_t)d.dst + (size_t)(d.H - 1) * d.dp + (size_t)d.W * es});
            ins.push_back({(uintptr_t)d.src, (uintptr_t)d.src + (size_t)(d.H - 1) * d.sp + (size_t)d.W * es});
        }
        std::vector<std::pair<uintptr_t, uintptr_t>> so = outs;
        std::sort(so.begin(), so.end());
        for (size_t k = 1; k < so.size(); ++k)
            if (so[k].first < so[k - 1].second) return ICL_ERR_ALIAS;
        std::sort(ins.begin(), ins.end());
        for (const auto& o : so) {
            auto it = std::lower_bound(ins.begin(), ins.end(), std::make_pair(o.second, (uintptr_t)0));
            // any input starting before o ends and ending after o starts overlaps
            for (auto j = ins.begin(); j != it; ++j)
                if (j->second > o.first) return ICL_ERR_ALIAS;
        }
    }
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    icl_batch_plan* p = new (std::nothrow) icl_batch_plan{};
    if (!p) return ICL_ERR_INVALID_VALUE;
    p->dt = dtype;
    p->nitems = (int)items.size();
    p->pixels = pixels;
    p->nimg = count;
    p->rmax = 0;
    for (const DevImage& d : imgs)
        if (d.src) p->rmax = std::max(p->rmax, d.r);
    p->tuned = -1;
    hipError_t e = hipSuccess;
    if (!imgs.empty()) e = hipMalloc(&p->d_imgs, imgs.size() * sizeof(DevImage));
    for (int w = 0; w < NWALKS; ++w) {
        p->ntiles[w] = (int)tiles[w].size();
        if (e == hipSuccess && !tiles[w].empty()) e = hipMalloc(&p->d_tiles[w], tiles[w].size() * sizeof(BatchTile));
        if (e == hipSuccess && !tiles[w].empty())
            e = hipMemcpy(p->d_tiles[w], tiles[w].data(), tiles[w].size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !items.empty()) e = hipMalloc(&p->d_items, items.size() * sizeof(StripItem));
    if (e == hipSuccess && !imgs.empty())
        e = hipMemcpy(p->d_imgs, imgs.data(), imgs.size() * sizeof(DevImage), hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(StripItem), hipMemcpyHostToDevice);
    p->col_ok = col_ok;
    for (int c = 0; c < NCOL; ++c) {
        p->ncol[c] = (int)cols[c].size();
        for (int r = 0; r <= RMAX; ++r) {   // items of radius r end after those of radius >= r
            int n = 0;
            for (const ColItem& it : cols[c]) n += imgs[it.img].r >= r ? 1 : 0;
            p->col_rg[c].end[r] = n;
        }
        if (e == hipSuccess && !cols[c].empty()) e = hipMalloc(&p->d_col[c], cols[c].size() * sizeof(ColItem));
        if (e == hipSuccess && !cols[c].empty())
            e = hipMemcpy(p->d_col[c], cols[c].data(), cols[c].size() * sizeof(ColItem), hipMemcpyHostToDevice);
    }
    int per_cu_col[2] = {};
    int per_cu[NWALKS] = {}, per_cu_strip = 0, dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int w = 0; w < NWALKS && e == hipSuccess; ++w)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[w], kernel_for(dtype, w), 256, 0);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_strip, strip_kernel_for(dtype), 64, 0);
    for (int cx = 1; cx <= 2 && e == hipSuccess; ++cx)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_col[cx - 1], col_kernel_for(dtype, cx), 256, 0);
    if (e != hipSuccess) {
        icl_batch_plan_destroy(p);
        return hip_status(e);
    }
    for (int c = 0; c < NCOL; ++c) {
        const long long resident = (long long)std::max(per_cu_col[kColCx[c] - 1], 1) * std::max(cus, 1);
        p->col_grid[c] = (int)std::min<long long>(resident, std::max(p->ncol[c], 1));
        if (p->col_grid[c] > 8) p->col_grid[c] -= p->col_grid[c] % 8;
    }
    for (int w = 0; w < NWALKS; ++w) {
        const long long resident = (long long)std::max(per_cu[w], 1) * std::max(cus, 1);
        p->grid[w] = (int)std::min<long long>(resident, std::max(p->ntiles[w], 1));
        // a multiple of 8 keeps the XCD-aware remap a permutation of the grid
        if (p->grid[w] > 8) p->grid[w] -= p->grid[w] % 8;
    }
    const long long resident_strip = (long long)std::max(per_cu_strip, 1) * std::max(cus, 1);
    p->strip_grid = (int)std::min<long long>(resident_strip, std::max(p->nitems, 1));
    *plan = p;
    return ICL_OK;
}

icl_status icl_conv_sep_batched(const icl_batch_plan* plan, void* stream) {
    if (!plan) return ICL_ERR_INVALID_VALUE;
    if (plan->ntiles[0] == 0) return ICL_OK;
    const int v = plan_variant(plan);
    if (v < 0 || v >= icl_variant_count(ICL_OP_CONV_SEP_BATCHED)) return ICL_ERR_UNSUPPORTED;
    return hip_status(launch_plan(plan, v, (hipStream_t)stream));
}

icl_status icl_batch_plan_variant(const icl_batch_plan* plan, int* index) {
    if (!plan || !index) return ICL_ERR_INVALID_VALUE;
    *index = plan_variant(plan);
    return ICL_OK;
}

icl_status icl_batch_plan_tune(icl_batch_plan* plan, void* stream) {
    if (!plan) return ICL_ERR_INVALID_VALUE;
    if (plan->ntiles[0] == 0) return ICL_OK;
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ICL_ERR_UNSUPPORTED;
    unsigned long long* d_h = nullptr;
    hipError_t e = hipMalloc(&d_h, sizeof(unsigned long long));
    if (e != hipSuccess) return hip_status(e);
    const int nv = icl_variant_count(ICL_OP_CONV_SEP_BATCHED);
    const int ref_v = batched_default();
    unsigned long long ref = 0;
    e = launch_plan(plan, ref_v, st);
    if (e == hipSuccess) e = plan_digest(plan, d_h, &ref, st);
    hipEvent_t ev[2];
    hipEventCreate(&ev[0]);
    hipEventCreate(&ev[1]);
    double best = 1e300;
    int best_v = -1;
    const bool log = std::getenv("ICL_LOG") && std::atoi(std::getenv("ICL_LOG")) >= 1;
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
        if (!variant_allowed(ICL_OP_CONV_SEP_BATCHED, v)) continue;
        unsigned long long h = 0;
        if ((e = launch_plan(plan, v, st)) != hipSuccess || (e = plan_digest(plan, d_h, &h, st)) != hipSuccess) break;
        if (h != ref) {   // every walk evaluates the same float32 expression: the outputs must match bit for bit
            if (log) std::fprintf(stderr, "icl tune: conv_sep_batched/%s rejected (output differs)\n",
                                  icl_variant_name(ICL_OP_CONV_SEP_BATCHED, v));
            continue;
        }
        constexpr int reps = 5, per = 4;
        std::vector<double> t;
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_plan(plan, v, st);
        for (int k = 0; k < reps && e == hipSuccess; ++k) {
            hipEventRecord(ev[0], st);
            for (int j = 0; j < per && e == hipSuccess; ++j) e = launch_plan(plan, v, st);
            hipEventRecord(ev[1], st);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            hipEventElapsedTime(&ms, ev[0], ev[1]);
            t.push_back(ms * 1000.0 / per);
        }
        if (e != hipSuccess) break;
        std::sort(t.begin(), t.end());
        const double us = t[t.size() / 2];
        if (log) std::fprintf(stderr, "icl tune: conv_sep_batched/%s %.2f us\n", icl_variant_name(ICL_OP_CONV_SEP_BATCHED, v), us);
        if (us < best) {
            best = us;
            best_v = v;
        }
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    hipFree(d_h);
    if (e != hipSuccess) return hip_status(e);
    if (best_v < 0) return ICL_ERR_UNSUPPORTED;
    plan->tuned = best_v;
    tune_cache_put(plan_problem(plan), best_v, best);
    return ICL_OK;
}

}  // extern "C"

namespace {

template <int CX, int STEP>
void launch_col(const icl_batch_plan* plan, int c, hipStream_t st) {
    switch (plan->dt) {
        case ICL_F32:
            hipLaunchKernelGGL((sep_batched_col_k<F32, CX, STEP>), dim3(plan->col_grid[c]), dim3(256), 0, st,
                               plan->d_imgs, plan->d_col[c], plan->col_rg[c]);
            break;
        case ICL_F16:
            hipLaunchKernelGGL((sep_batched_col_k<F16, CX, STEP>), dim3(plan->col_grid[c]), dim3(256), 0, st,
                               plan->d_imgs, plan->d_col[c], plan->col_rg[c]);
            break;
        default:
            hipLaunchKernelGGL((sep_batched_col_k<BF16, CX, STEP>), dim3(plan->col_grid[c]), dim3(256), 0, st,
                               plan->d_imgs, plan->d_col[c], plan->col_rg[c]);
            break;
    }
}

hipError_t launch_plan(const icl_batch_plan* plan, int v, hipStream_t st) {
    if (v >= kFirstCol) {
        const int c = v - kFirstCol;
        if (!plan->col_ok) return hipErrorInvalidValue;
        if (kColCx[c] == 1) launch_col<1, 64>(plan, c, st);
        else launch_col<2, 32>(plan, c, st);
        return hipGetLastError();
    }
    if (v == 1) {
        switch (plan->dt) {
            case ICL_F32:
                hipLaunchKernelGGL(sep_batched_strip_k<F32>, dim3(plan->strip_grid), dim3(64), 0, st, plan->d_imgs,
                                   plan->d_items, plan->nitems);
                break;
            case ICL_F16:
                hipLaunchKernelGGL(sep_batched_strip_k<F16>, dim3(plan->strip_grid), dim3(64), 0, st, plan->d_imgs,
                                   plan->d_items, plan->nitems);
                break;
            default:
                hipLaunchKernelGGL(sep_batched_strip_k<BF16>, dim3(plan->strip_grid), dim3(64), 0, st, plan->d_imgs,
                                   plan->d_items, plan->nitems);
                break;
        }
        return hipGetLastError();
    }
    const int w = v == 0 ? 0 : v - 1;   // variants 0, 2, 3 are tile walks 0, 1, 2
    switch (plan->dt) {
        case ICL_F32: launch_walk<F32>(plan, w, st); break;
        case ICL_F16: launch_walk<F16>(plan, w, st); break;
        default: launch_walk<BF16>(plan, w, st); break;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

icl_status icl_batch_plan_info(const icl_batch_plan* plan, long long* tiles, long long* pixels) {
    if (!plan) return ICL_ERR_INVALID_VALUE;
    if (tiles) *tiles = plan->ntiles[0];
    if (pixels) *pixels = plan->pixels;
    return ICL_OK;
}

void icl_batch_plan_destroy(icl_batch_plan* plan) {
    if (!plan) return;
    hipFree(plan->d_imgs);
    for (int w = 0; w < NWALKS; ++w) hipFree(plan->d_tiles[w]);
    hipFree(plan->d_items);
    for (int c = 0; c < NCOL; ++c) hipFree(plan->d_col[c]);
    delete plan;
}

icl_status icl_batch_graph_create(const icl_batch_plan* plan, void** exec) {
    if (!plan || !exec) return ICL_ERR_INVALID_VALUE;
    *exec = nullptr;
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_status(e);
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const icl_status ls = icl_conv_sep_batched(plan, st);
        const hipError_t ee = hipStreamEndCapture(st, &graph);
        if (ls != ICL_OK) {
            if (graph) hipGraphDestroy(graph);
            hipStreamDestroy(st);
            return ls;
        }
        e = ee;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(st);
    if (e != hipSuccess) return hip_status(e);
    *exec = ge;
    return ICL_OK;
}

icl_status icl_graph_launch(void* exec, void* stream) {
    if (!exec) return ICL_ERR_INVALID_VALUE;
    return hip_status(hipGraphLaunch((hipGraphExec_t)exec, (hipStream_t)stream));
}

void icl_graph_destroy(void* exec) {
    if (exec) hipGraphExecDestroy((hipGraphExec_t)exec);
}

}  // extern "C"
