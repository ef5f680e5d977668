// Auto-tuner: picks, per device and problem class, the fastest precompiled
// variant of an operation (the paper's auto-tuner, Section 4: run candidate
// implementations, time them, keep the best; its discussion notes that only
// valid candidates count and that compilation dominated its tuning time - here
// every candidate is compiled ahead of time, so a search costs run time only).
//
// Search: every variant that supports the problem runs once on synthetic data
// and its output is compared with the plain variant's (a candidate that
// disagrees is rejected); the survivors are timed with HIP events over a set of
// rotating buffers (>= 1 GiB in total where the problem allows, so the 256 MB
// Infinity Cache cannot hold the working set), and the median decides.
//
// Cache: key = gfx arch | CU count | op | dtype | radius | size class
// (floor(log2(pixels))), value = variant NAME (so a rebuilt library with a
// different table never maps an entry onto the wrong kernel) and its time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "icl_device.hpp"
#include "icl_internal.hpp"

namespace icl {
namespace {

struct Entry {
    std::string variant;
    double us;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;
std::string g_device_tag;   // "gfx950|256"

const std::string& device_tag() {
    if (g_device_tag.empty()) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            std::string arch(prop.gcnArchName);
            const size_t c = arch.find(':');
            if (c != std::string::npos) arch = arch.substr(0, c);
            g_device_tag = arch + "|" + std::to_string(prop.multiProcessorCount);
        } else {
            g_device_tag = "unknown|0";
        }
    }
    return g_device_tag;
}

int size_class(int W, int H) {
    const double px = std::max(1.0, (double)W * (double)H);
    return (int)std::floor(std::log2(px));
}

std::string make_key(icl_op op, icl_dtype dt, int r, int W, int H) {
    return device_tag() + "|" + op_name(op) + "|" + std::to_string((int)dt) + "|" + std::to_string(r) + "|" +
           std::to_string(size_class(W, H));
}

int index_of(icl_op op, const std::string& name) {
    const int n = icl_variant_count(op);
    for (int i = 0; i < n; ++i)
        if (name == icl_variant_name(op, i)) return i;
    return -1;
}

std::string default_cache_path() {
    if (const char* p = std::getenv("ICL_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : ".") + "/.cache/icl/tune.json";
}

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ float hash_uniform(unsigned long long i, unsigned long long seed) {
    unsigned long long z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)(z >> 40) * (1.0f / 16777216.0f);
}

template <class T>
__global__ void fill_k(void* dst, size_t pitch, int W, int H, unsigned long long seed) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)W * H) return;
    const int y = (int)(i / W), x = (int)(i % W);
    store_px<T>(dst, (size_t)y * pitch + (size_t)x * T::size, hash_uniform(i, seed));
}

// out[0] = max |a - b|, out[1] = max |b| (as float bits; values are non-negative).
// Each block reduces in LDS first, so only one pair of atomics per block reaches memory.
template <class T>
__global__ __launch_bounds__(256) void compare_k(const void* a, const void* b, size_t pitch, int W, int H,
                                                 unsigned* out) {
    __shared__ unsigned red[2][256];
    const size_t n = (size_t)W * H;
    unsigned md = 0, mb = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int y = (int)(i / W), x = (int)(i % W);
        const size_t off = (size_t)y * pitch + (size_t)x * T::size;
        const float va = load_px<T>(a, off), vb = load_px<T>(b, off);
        float d = fabsf(va - vb);
        if (!(d == d)) d = 3.0e38f;   // NaN counts as a mismatch
        md = max(md, __float_as_uint(d));
        mb = max(mb, __float_as_uint(fabsf(vb)));
    }
    red[0][threadIdx.x] = md;
    red[1][threadIdx.x] = mb;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = max(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], red[0][0]);
        atomicMax(&out[1], red[1][0]);
    }
}

__global__ void compare_u8_k(const uint8_t* a, const uint8_t* b, size_t pitch, int W, int H, unsigned* out) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)W * H) return;
    const int y = (int)(i / W), x = (int)(i % W);
    if (a[(size_t)y * pitch + x] != b[(size_t)y * pitch + x]) atomicAdd(&out[0], 1u);
}

__global__ void fill_u8_k(uint8_t* p, size_t pitch, int W, int H, unsigned long long seed) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)W * H) return;
    const int y = (int)(i / W), x = (int)(i % W);
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    p[(size_t)y * pitch + x] = (uint8_t)((z ^ (z >> 31)) >> 56);
}

__global__ void zero2_k(unsigned* p) {
    if (threadIdx.x < 2) p[threadIdx.x] = 0u;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

hipError_t fill(icl_dtype dt, void* p, size_t pitch, int W, int H, unsigned long long seed, hipStream_t st) {
    const unsigned nb = blocks_for((size_t)W * H);
    switch (dt) {
        case ICL_F32: hipLaunchKernelGGL(fill_k<F32>, dim3(nb), dim3(256), 0, st, p, pitch, W, H, seed); break;
        case ICL_F16: hipLaunchKernelGGL(fill_k<F16>, dim3(nb), dim3(256), 0, st, p, pitch, W, H, seed); break;
        default: hipLaunchKernelGGL(fill_k<BF16>, dim3(nb), dim3(256), 0, st, p, pitch, W, H, seed); break;
    }
    return hipGetLastError();
}

// true when a matches b to within rel * max|b| (+ a tiny absolute floor)
bool outputs_agree(icl_dtype dt, const void* a, const void* b, size_t pitch, int W, int H, unsigned* d_stat,
                   hipStream_t st) {
    hipLaunchKernelGGL(zero2_k, dim3(1), dim3(64), 0, st, d_stat);
    const unsigned nb = std::min(blocks_for((size_t)W * H), 2048u);
    switch (dt) {
        case ICL_F32: hipLaunchKernelGGL(compare_k<F32>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
        case ICL_F16: hipLaunchKernelGGL(compare_k<F16>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
        default: hipLaunchKernelGGL(compare_k<BF16>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
    }
    unsigned h[2] = {0, 0};
    if (hipMemcpyAsync(h, d_stat, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    if (hipStreamSynchronize(st) != hipSuccess) return false;
    float maxd, maxb;
    std::memcpy(&maxd, &h[0], 4);
    std::memcpy(&maxb, &h[1], 4);
    const float rel = dt == ICL_F32 ? 1e-4f : 1e-2f;
    return maxd <= rel * maxb + 1e-6f;
}

bool masks_agree(const uint8_t* a, const uint8_t* b, size_t pitch, int W, int H, unsigned* d_stat, hipStream_t st) {
    hipLaunchKernelGGL(zero2_k, dim3(1), dim3(64), 0, st, d_stat);
    hipLaunchKernelGGL(compare_u8_k, dim3(blocks_for((size_t)W * H)), dim3(256), 0, st, a, b, pitch, W, H, d_stat);
    unsigned h = 1;
    if (hipMemcpyAsync(&h, d_stat, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    if (hipStreamSynchronize(st) != hipSuccess) return false;
    return h == 0;
}

// Per-launch time (us): after `warm` launches, `reps` event-bracketed batches of `per`
// back-to-back launches (rotating over `sets` buffer sets); the median batch mean wins.
// Batches amortise the dispatch gap that a per-launch event pair would add.
template <class F>
double time_launches(F&& launch, int sets, int warm, int reps, int per, hipStream_t st, bool* ok) {
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev) hipEventCreate(&e);
    *ok = true;
    int k = 0;
    for (int i = 0; i < warm; ++i)
        if (launch(k++ % sets) != hipSuccess) *ok = false;
    for (int i = 0; i < reps; ++i) {
        hipEventRecord(ev[2 * i], st);
        for (int j = 0; j < per; ++j)
            if (launch(k++ % sets) != hipSuccess) *ok = false;
        hipEventRecord(ev[2 * i + 1], st);
    }
    hipStreamSynchronize(st);
    std::vector<double> t;
    for (int i = 0; i < reps; ++i) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        t.push_back(ms * 1000.0 / per);
    }
    for (auto& e : ev) hipEventDestroy(e);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

int rotation_sets(size_t bytes_per_set) {
    const size_t target = (size_t)1 << 30;
    size_t k = (target + bytes_per_set - 1) / std::max<size_t>(bytes_per_set, 1);
    return (int)std::min<size_t>(std::max<size_t>(k, 2), 8);
}

bool log_on() {
    const char* lv = std::getenv("ICL_LOG");
    return lv && std::atoi(lv) >= 1;
}

struct Buffers {
    std::vector<void*> ptrs;
    ~Buffers() {
        for (void* p : ptrs) hipFree(p);
    }
    void* alloc(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 256)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

// How a search explores the candidates: every one (exhaustive), or the paper's model-guided
// search (Section 4): time `samples` random candidates, fit the time model, time the `top_k`
// best-predicted of the rest, keep the fastest measured.
struct SearchPlan {
    bool model = false;
    int samples = 0, top_k = 0;
    unsigned long long seed = 0;
    int timed = 0;   // out: candidates timed
};
thread_local SearchPlan g_plan;

// Generic search over an op's variant table.  make(set) builds the argument bundle
// for buffer set `set`; agree(a) checks a candidate's output (set 0) against the
// plain output.
template <class A, class Make, class Agree>
icl_status search(icl_op op, const Variant<A>* tab, int count, icl_dtype dt, int r, int W, int H, int sets,
                  Make&& make, Agree&& agree, hipStream_t st) {
    double best = 1e300;
    int best_i = -1;
    std::vector<double> measured(count, -1.0);   // us, -1 = not timed, -2 = rejected
    auto try_one = [&](int i) {
        const A a0 = make(0, i);
        measured[i] = -2.0;
        if (tab[i].launch(a0) != hipSuccess) return;
        if (!agree()) {
            if (log_on()) std::fprintf(stderr, "icl tune: %s/%s rejected (output differs from plain)\n", op_name(op),
                                       tab[i].name);
            return;
        }
        bool ok = true;
        const double us = time_launches([&](int s) { return tab[i].launch(make(s, i)); }, sets, 3, 5, 8, st, &ok);
        ++g_plan.timed;
        if (!ok) return;
        measured[i] = us;
        if (log_on()) std::fprintf(stderr, "icl tune: %s/%s %.2f us\n", op_name(op), tab[i].name, us);
        if (us < best) {
            best = us;
            best_i = i;
        }
    };
    std::vector<int> cand;
    for (int i = 1; i < count; ++i)
        if (tab[i].supports(make(0, i))) cand.push_back(i);
    g_plan.timed = 0;
    const int ns = std::max(2, g_plan.samples);
    if (!g_plan.model || (int)cand.size() <= ns + std::max(1, g_plan.top_k)) {
        for (int i : cand) try_one(i);   // exhaustive (also when the model would time everything anyway)
    } else {
        // random sample (Fisher-Yates on a SplitMix64 stream)
        uint64_t s = g_plan.seed;
        std::vector<int> order = cand;
        for (int i = (int)order.size() - 1; i > 0; --i) {
            uint64_t z = (s += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            std::swap(order[i], order[(int)(z % (uint64_t)(i + 1))]);
        }
        for (int k = 0; k < ns; ++k) try_one(order[k]);
        std::vector<std::string> names;
        for (int i = 0; i < count; ++i) names.push_back(tab[i].name);
        std::vector<std::vector<double>> F;
        variant_features(names, F);
        std::vector<std::vector<double>> X;
        std::vector<double> y;
        for (int i : cand)
            if (measured[i] > 0) {
                X.push_back(F[i]);
                y.push_back(std::log(measured[i]));
            }
        PerfModel m;
        std::vector<std::pair<double, int>> pred;
        if ((int)X.size() >= 2 && m.fit(X, y, 8, 2000, g_plan.seed ^ 0x5bd1e995ull)) {
            for (int i : cand)
                if (measured[i] == -1.0) pred.push_back({m.predict(F[i]), i});
            std::sort(pred.begin(), pred.end());
            for (int k = 0; k < (int)pred.size() && k < g_plan.top_k; ++k) try_one(pred[k].second);
        } else {
            for (int i : cand)
                if (measured[i] == -1.0) try_one(i);
        }
    }
    if (best_i < 0) return ICL_ERR_UNSUPPORTED;
    tune_cache_put(op, dt, r, W, H, best_i, best);
    return ICL_OK;
}

icl_status tune_conv(icl_op op, icl_dtype dt, int r, int W, int H, hipStream_t st) {
    const int es = elem_size(dt);
    const size_t pitch = ((size_t)W * es + 255) & ~(size_t)255;
    const size_t bytes = pitch * H;
    const int sets = rotation_sets(2 * bytes);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(bytes);
        dst[s] = b.alloc(bytes);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        if (fill(dt, src[s], pitch, W, H, 0x1234ull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(bytes);
    const int n = 2 * r + 1;
    const int ntaps = op == ICL_OP_CONV2D ? n * n : 2 * n;
    std::vector<float> taps(ntaps);
    double sum = 0;
    for (int k = 0; k < ntaps; ++k) sum += (taps[k] = 1.0f + 0.25f * (float)((k * 7) % 5));
    const double norm = op == ICL_OP_CONV2D ? sum : sum / 2.0;   // each separable pass sums to 1
    for (auto& t : taps) t = (float)(t / norm);
    float* d_taps = static_cast<float*>(b.alloc(ntaps * sizeof(float)));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    void* ws = op == ICL_OP_CONV_SEP ? b.alloc(sep_workspace(W, H)) : nullptr;
    if (!ref || !d_taps || !d_stat || (op == ICL_OP_CONV_SEP && !ws)) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_taps, taps.data(), ntaps * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
        return ICL_ERR_HIP;
    if (op == ICL_OP_CONV_SEP) {
        int count;
        const Variant<SepArgs>* tab = sep_variants(&count);
        auto make = [&](int s, int) {
            return SepArgs{src[s], pitch, dst[s], pitch, W, H, dt, d_taps, d_taps + n, r, ws, sep_workspace(W, H), st};
        };
        SepArgs p0 = make(0, 0);
        p0.dst = ref;
        if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
        auto agree = [&]() { return outputs_agree(dt, dst[0], ref, pitch, W, H, d_stat, st); };
        return search(op, tab, count, dt, r, W, H, sets, make, agree, st);
    } else {
        int count;
        const Variant<Conv2dArgs>* tab = conv2d_variants(&count);
        auto make = [&](int s, int) { return Conv2dArgs{src[s], pitch, dst[s], pitch, W, H, dt, d_taps, r, st}; };
        Conv2dArgs p0 = make(0, 0);
        p0.dst = ref;
        if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
        auto agree = [&]() { return outputs_agree(dt, dst[0], ref, pitch, W, H, d_stat, st); };
        return search(op, tab, count, dt, r, W, H, sets, make, agree, st);
    }
}

icl_status tune_harris(int rg, int W, int H, hipStream_t st) {
    const size_t pitch = ((size_t)W * 4 + 255) & ~(size_t)255;
    const size_t bytes = pitch * H;
    const int sets = rotation_sets(2 * bytes);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(bytes);
        dst[s] = b.alloc(bytes);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        if (fill(ICL_F32, src[s], pitch, W, H, 0x777ull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(bytes);
    const int n = 2 * rg + 1;
    std::vector<float> g(n);
    double sum = 0;
    for (int k = 0; k < n; ++k) sum += (g[k] = std::exp(-0.5f * (float)((k - rg) * (k - rg))));
    for (auto& v : g) v = (float)(v / sum);
    float* d_g = static_cast<float*>(b.alloc(n * sizeof(float)));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    void* ws = b.alloc(harris_workspace(W, H));
    if (!ref || !d_g || !d_stat || !ws) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_g, g.data(), n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess) return ICL_ERR_HIP;
    int count;
    const Variant<HarrisArgs>* tab = harris_variants(&count);
    auto make = [&](int s, int) {
        return HarrisArgs{static_cast<const float*>(src[s]), pitch, static_cast<float*>(dst[s]), pitch, W, H, d_g, rg,
                          0.04f, ws, harris_workspace(W, H), st};
    };
    HarrisArgs p0 = make(0, 0);
    p0.resp = static_cast<float*>(ref);
    if (tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    auto agree = [&]() { return outputs_agree(ICL_F32, dst[0], ref, pitch, W, H, d_stat, st); };
    return search(ICL_OP_HARRIS, tab, count, ICL_F32, rg, W, H, sets, make, agree, st);
}

icl_status tune_conv_u8(int r, int W, int H, hipStream_t st) {
    const size_t pitch = ((size_t)W + 255) & ~(size_t)255;
    const int sets = rotation_sets(2 * pitch * H);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(pitch * H);
        dst[s] = b.alloc(pitch * H);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        hipLaunchKernelGGL(fill_u8_k, dim3(blocks_for((size_t)W * H)), dim3(256), 0, st,
                           static_cast<uint8_t*>(src[s]), pitch, W, H, 0x77ull + s);
        if (hipGetLastError() != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(pitch * H);
    const int n = 2 * r + 1;
    std::vector<int16_t> taps(n * n);
    for (int k = 0; k < n * n; ++k) taps[k] = (int16_t)(160 + 97 * ((k * 7) % 5) - 40 * (k % 3));
    int16_t* d_taps = static_cast<int16_t*>(b.alloc(taps.size() * sizeof(int16_t)));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    if (!ref || !d_taps || !d_stat) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_taps, taps.data(), taps.size() * sizeof(int16_t), hipMemcpyHostToDevice, st) != hipSuccess)
        return ICL_ERR_HIP;
    int count;
    const Variant<U8Args>* tab = conv2d_u8_variants(&count);
    const int shift = 12;
    auto make = [&](int s, int) {
        return U8Args{static_cast<const uint8_t*>(src[s]), pitch, static_cast<uint8_t*>(dst[s]), pitch, W, H, d_taps,
                      r, shift, 0, 0, st};
    };
    U8Args p0 = make(0, 0);
    p0.dst = static_cast<uint8_t*>(ref);
    if (tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    auto agree = [&]() {   // integer results: every variant must return the same bytes
        return masks_agree(static_cast<uint8_t*>(dst[0]), static_cast<uint8_t*>(ref), pitch, W, H, d_stat, st);
    };
    return search(ICL_OP_CONV2D_U8, tab, count, ICL_U8, r, W, H, sets, make, agree, st);
}

// Fused corners: the single-pass variants share their arithmetic, so each must return the
// default single-pass variant's mask byte for byte (the two-kernel variant is not a candidate).
icl_status tune_corners(int rg, int W, int H, hipStream_t st) {
    const size_t pitch = ((size_t)W * 4 + 255) & ~(size_t)255;
    const size_t mpitch = ((size_t)W + 255) & ~(size_t)255;
    const int sets = rotation_sets(pitch * H + mpitch * H);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(pitch * H);
        dst[s] = b.alloc(mpitch * H);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        if (fill(ICL_F32, src[s], pitch, W, H, 0x55ull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(mpitch * H);
    const int n = 2 * rg + 1;
    std::vector<float> g(n);
    double sum = 0;
    for (int i = 0; i < n; ++i) sum += (g[i] = 1.0f + (float)(rg - std::abs(i - rg)));
    for (auto& t : g) t = (float)(t / sum);
    float* d_g = static_cast<float*>(b.alloc(n * sizeof(float)));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    if (!ref || !d_g || !d_stat) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_g, g.data(), n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess) return ICL_ERR_HIP;
    int count;
    const Variant<CornersArgs>* tab = corners_variants(&count);
    auto make = [&](int s, int) {
        return CornersArgs{static_cast<const float*>(src[s]), pitch, static_cast<uint8_t*>(dst[s]), mpitch, W, H,
                           d_g, rg, 0.04f, 1, 1e-6f, nullptr, 0, nullptr, 0, st};
    };
    CornersArgs p0 = make(0, 0);
    p0.M = static_cast<uint8_t*>(ref);
    const int deflt = corners_default(p0);
    if (deflt == 0 || !tab[deflt].supports(p0) || tab[deflt].launch(p0) != hipSuccess) return ICL_ERR_UNSUPPORTED;
    auto agree = [&]() {
        return masks_agree(static_cast<uint8_t*>(dst[0]), static_cast<uint8_t*>(ref), mpitch, W, H, d_stat, st);
    };
    return search(ICL_OP_CORNERS, tab, count, ICL_F32, rg, W, H, sets, make, agree, st);
}

icl_status tune_nms(int r, int W, int H, hipStream_t st) {
    const size_t pitch = ((size_t)W * 4 + 255) & ~(size_t)255;
    const size_t mpitch = ((size_t)W + 255) & ~(size_t)255;
    const int sets = rotation_sets(pitch * H + mpitch * H);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(pitch * H);
        dst[s] = b.alloc(mpitch * H);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        if (fill(ICL_F32, src[s], pitch, W, H, 0x99ull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(mpitch * H);
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    if (!ref || !d_stat) return ICL_ERR_HIP;
    int count;
    const Variant<NmsArgs>* tab = nms_variants(&count);
    auto make = [&](int s, int) {
        return NmsArgs{static_cast<const float*>(src[s]), pitch, static_cast<uint8_t*>(dst[s]), mpitch, W, H, r,
                       0.5f, st};
    };
    NmsArgs p0 = make(0, 0);
    p0.M = static_cast<uint8_t*>(ref);
    if (tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    auto agree = [&]() {
        return masks_agree(static_cast<uint8_t*>(dst[0]), static_cast<uint8_t*>(ref), mpitch, W, H, d_stat, st);
    };
    return search(ICL_OP_NMS, tab, count, ICL_F32, r, W, H, sets, make, agree, st);
}

// ------------------------------------------------------------------ tiny JSON reader for our own cache file
bool parse_cache(const std::string& text, std::map<std::string, Entry>& out) {
    // format: {"version": 1, "entries": [{"key": "...", "variant": "...", "us": 1.0}, ...]}
    if (text.find("\"version\": 1") == std::string::npos) return false;
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return false;
    auto str_field = [&](size_t from, const char* name, size_t limit, std::string& v) -> bool {
        const std::string pat = std::string("\"") + name + "\": \"";
        const size_t p = text.find(pat, from);
        if (p == std::string::npos || p > limit) return false;
        const size_t s = p + pat.size();
        const size_t e = text.find('"', s);
        if (e == std::string::npos || e > limit) return false;
        v = text.substr(s, e - s);
        return true;
    };
    while (true) {
        const size_t ob = text.find('{', pos + 1);
        if (ob == std::string::npos) break;
        const size_t cb = text.find('}', ob);
        if (cb == std::string::npos) return false;
        std::string key, var;
        if (!str_field(ob, "key", cb, key) || !str_field(ob, "variant", cb, var)) return false;
        const size_t up = text.find("\"us\": ", ob);
        double us = 0;
        if (up != std::string::npos && up < cb) us = std::atof(text.c_str() + up + 6);
        out[key] = Entry{var, us};
        pos = cb;
    }
    return true;
}

}  // namespace

void tune_cache_put(icl_op op, icl_dtype dt, int r, int W, int H, int variant, double us) {
    const char* name = icl_variant_name(op, variant);
    if (!name) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[make_key(op, dt, r, W, H)] = Entry{name, us};
}

int tune_cache_get(icl_op op, icl_dtype dt, int r, int W, int H) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_cache.empty()) return -1;
    auto it = g_cache.find(make_key(op, dt, r, W, H));
    if (it == g_cache.end()) return -1;
    return index_of(op, it->second.variant);
}

}  // namespace icl

using namespace icl;

extern "C" {

icl_status icl_tune_model(icl_op op, icl_dtype dtype, int radius, int width, int height, int samples, int top_k,
                          unsigned long long seed, int* timed, void* stream) {
    if (samples < 2 || top_k < 1) return ICL_ERR_INVALID_VALUE;
    g_plan = SearchPlan{true, samples, top_k, seed, 0};
    const icl_status s = icl_tune(op, dtype, radius, width, height, stream);
    g_plan.model = false;
    if (timed) *timed = g_plan.timed;
    return s;
}

icl_status icl_tune(icl_op op, icl_dtype dtype, int radius, int width, int height, void* stream) {
    if (width < 1 || height < 1) return ICL_ERR_INVALID_VALUE;
    if (op == ICL_OP_CONV2D_U8 ? dtype != ICL_U8 : (dtype != ICL_F32 && dtype != ICL_F16 && dtype != ICL_BF16))
        return ICL_ERR_DTYPE;
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ICL_ERR_UNSUPPORTED;
    switch (op) {
        case ICL_OP_CONV_SEP:
        case ICL_OP_CONV2D:
            if (radius < 0 || radius > ICL_MAX_RADIUS) return ICL_ERR_RADIUS;
            s = tune_conv(op, dtype, radius, width, height, st);
            break;
        case ICL_OP_HARRIS:
            if (radius < 0 || radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            s = tune_harris(radius, width, height, st);
            break;
        case ICL_OP_CORNERS:
            if (radius < 0 || radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            if (radius > 3) return ICL_OK;   // only the two-kernel variant: nothing to choose
            s = tune_corners(radius, width, height, st);
            break;
        case ICL_OP_CONV2D_U8:
            if (radius < 0 || radius > ICL_MAX_U8_RADIUS) return ICL_ERR_RADIUS;
            s = tune_conv_u8(radius, width, height, st);
            break;
        case ICL_OP_NMS:
            if (radius < 1 || radius > ICL_MAX_NMS_RADIUS) return ICL_ERR_RADIUS;
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            s = tune_nms(radius, width, height, st);
            break;
        case ICL_OP_CONV_SEP_BATCHED: case ICL_OP_BANK_FWD: case ICL_OP_BANK_BWD_INPUT: case ICL_OP_BANK_BWD_FILTER:
        case ICL_OP_SSE_LOSS:
            return ICL_OK;   // a single variant: nothing to choose
        default: return ICL_ERR_INVALID_VALUE;
    }
    hipStreamSynchronize(st);
    return s;
}

icl_status icl_tune_save(const char* path) {
    const std::string p = path ? std::string(path) : default_cache_path();
    const size_t slash = p.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // create parent directories one level at a time
        for (size_t q = p.find('/', 1); q != std::string::npos && q <= slash; q = p.find('/', q + 1))
            mkdir(p.substr(0, q).c_str(), 0755);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    FILE* f = std::fopen(p.c_str(), "w");
    if (!f) return ICL_ERR_TUNE_CACHE;
    std::fprintf(f, "{\"version\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : g_cache) {
        std::fprintf(f, "%s\n  {\"key\": \"%s\", \"variant\": \"%s\", \"us\": %.3f}", first ? "" : ",", kv.first.c_str(),
                     kv.second.variant.c_str(), kv.second.us);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? ICL_OK : ICL_ERR_TUNE_CACHE;
}

icl_status icl_tune_load(const char* path) {
    const std::string p = path ? std::string(path) : default_cache_path();
    FILE* f = std::fopen(p.c_str(), "r");
    if (!f) return ICL_ERR_TUNE_CACHE;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    std::map<std::string, Entry> parsed;
    if (!parse_cache(text, parsed)) return ICL_ERR_TUNE_CACHE;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : parsed) g_cache[kv.first] = kv.second;
    return ICL_OK;
}

void icl_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}

}  // extern "C"
