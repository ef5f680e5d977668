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
#include <new>
#include <vector>

#include "icl_device.hpp"
#include "icl_internal.hpp"
#include "sep_strip.hpp"
#include "sep_tile.hpp"
#include "tile_stage.hpp"

namespace icl {

struct DevImage {
    const void* src;
    void* dst;
    unsigned long long sp, dp;
    const float* tx;
    const float* ty;
    int W, H, r, vec_ok, vec_out, pad;
};

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

struct icl_batch_plan {
    icl_dtype dt;
    DevImage* d_imgs;
    BatchTile* d_tiles[NWALKS];
    int ntiles[NWALKS];
    int grid[NWALKS];
    StripItem* d_items;
    int nitems;
    int strip_grid;
    long long pixels;
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

const void* strip_kernel_for(icl_dtype dt) {
    switch (dt) {
        case ICL_F32: return reinterpret_cast<const void*>(&sep_batched_strip_k<F32>);
        case ICL_F16: return reinterpret_cast<const void*>(&sep_batched_strip_k<F16>);
        default: return reinterpret_cast<const void*>(&sep_batched_strip_k<BF16>);
    }
}

bool ranges_overlap(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) { return a0 < b1 && b0 < a1; }

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
        di.pad = 0;
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
    int per_cu[NWALKS] = {}, per_cu_strip = 0, dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int w = 0; w < NWALKS && e == hipSuccess; ++w)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[w], kernel_for(dtype, w), 256, 0);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_strip, strip_kernel_for(dtype), 64, 0);
    if (e != hipSuccess) {
        hipFree(p->d_imgs);
        for (int w = 0; w < NWALKS; ++w) hipFree(p->d_tiles[w]);
        hipFree(p->d_items);
        delete p;
        return hip_status(e);
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
    hipStream_t st = (hipStream_t)stream;
    const int v = select_variant(ICL_OP_CONV_SEP_BATCHED, plan->dt, 0, 0, 0, batched_default());
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
        return hip_status(hipGetLastError());
    }
    const int w = v == 0 ? 0 : v - 1;   // variants 0, 2, 3 are tile walks 0, 1, 2
    switch (plan->dt) {
        case ICL_F32: launch_walk<F32>(plan, w, st); break;
        case ICL_F16: launch_walk<F16>(plan, w, st); break;
        default: launch_walk<BF16>(plan, w, st); break;
    }
    return hip_status(hipGetLastError());
}

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
