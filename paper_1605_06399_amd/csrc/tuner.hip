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

int size_class(const Problem& p) {
    const double px = std::max(1.0, (double)p.W * (double)p.H * (double)std::max(p.D, 1) * (double)std::max(p.N, 1));
    return (int)std::floor(std::log2(px));
}

// device | op | dtype | radius | size class | filters | arithmetic mode
std::string make_key(const Problem& p) {
    return device_tag() + "|" + op_name(p.op) + "|" + std::to_string((int)p.dt) + "|" + std::to_string(p.r) + "|" +
           std::to_string(size_class(p)) + "|f" + std::to_string(std::max(p.F, 1)) + "|m" +
           std::to_string(math_mode());
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

// out[0] = max |a - b|, out[1] = max |b|, out[2] = max |a - b| / |b| (as float bits; values
// are non-negative, so the bit patterns order like the values).  Each block reduces in LDS
// first, so only one set of atomics per block reaches memory.
template <class T>
__global__ __launch_bounds__(256) void compare_k(const void* a, const void* b, size_t pitch, int W, int H,
                                                 unsigned* out) {
    __shared__ unsigned red[3][256];
    const size_t n = (size_t)W * H;
    unsigned md = 0, mb = 0, mr = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int y = (int)(i / W), x = (int)(i % W);
        const size_t off = (size_t)y * pitch + (size_t)x * T::size;
        const float va = load_px<T>(a, off), vb = load_px<T>(b, off);
        float d = fabsf(va - vb);
        if (!(d == d)) d = 3.0e38f;   // NaN counts as a mismatch
        float rel = d / fmaxf(fabsf(vb), 1e-30f);
        if (!(rel <= 3.0e38f)) rel = 3.0e38f;
        md = max(md, __float_as_uint(d));
        mb = max(mb, __float_as_uint(fabsf(vb)));
        mr = max(mr, __float_as_uint(rel));
    }
    red[0][threadIdx.x] = md;
    red[1][threadIdx.x] = mb;
    red[2][threadIdx.x] = mr;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = max(red[q][threadIdx.x], red[q][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], red[0][0]);
        atomicMax(&out[1], red[1][0]);
        atomicMax(&out[2], red[2][0]);
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
    if (threadIdx.x < 4) p[threadIdx.x] = 0u;
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

// Storage-type tolerance of the candidate check: the float32 normwise contract (1e-5) for
// float32, one output rounding for the half formats (a binary16 ulp is 2^-10 relative, a
// bfloat16 ulp 2^-7).
float storage_tol(icl_dtype dt) { return dt == ICL_F32 ? 1e-5f : (dt == ICL_F16 ? 2e-3f : 1e-2f); }

// How a candidate's output is compared with the reference output.
enum class Agree {
    PerPixel,   // |a - b| <= tol |b| at every pixel: the normwise error of a filter with non-negative
                // taps on non-negative data (the tuner's inputs), where S(p) is the exact output itself
    Max         // max |a - b| <= tol max |b|: for outputs with cancellation (the Harris response)
};

bool outputs_agree(icl_dtype dt, const void* a, const void* b, size_t pitch, int W, int H, unsigned* d_stat,
                   hipStream_t st, Agree how = Agree::PerPixel, float tol = 0.f) {
    hipLaunchKernelGGL(zero2_k, dim3(1), dim3(64), 0, st, d_stat);
    const unsigned nb = std::min(blocks_for((size_t)W * H), 2048u);
    switch (dt) {
        case ICL_F32: hipLaunchKernelGGL(compare_k<F32>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
        case ICL_F16: hipLaunchKernelGGL(compare_k<F16>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
        default: hipLaunchKernelGGL(compare_k<BF16>, dim3(nb), dim3(256), 0, st, a, b, pitch, W, H, d_stat); break;
    }
    unsigned h[3] = {0, 0, 0};
    if (hipMemcpyAsync(h, d_stat, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    if (hipStreamSynchronize(st) != hipSuccess) return false;
    float maxd, maxb, maxr;
    std::memcpy(&maxd, &h[0], 4);
    std::memcpy(&maxb, &h[1], 4);
    std::memcpy(&maxr, &h[2], 4);
    if (tol <= 0.f) tol = storage_tol(dt);
    if (how == Agree::PerPixel) return maxr <= tol;
    return maxd <= tol * maxb;
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
    if (bytes_per_set >= target) return 1;   // one set already exceeds the Infinity Cache fourfold
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
template <class A, class Make, class AgreeFn>
icl_status search(const Problem& pb, const Variant<A>* tab, int count, int sets, Make&& make, AgreeFn&& agree,
                  hipStream_t st) {
    const icl_op op = pb.op;
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
    // every variant but the reference (index 0) that runs the problem under the arithmetic mode
    std::vector<int> cand;
    for (int i = 1; i < count; ++i)
        if (variant_allowed(op, i) && tab[i].supports(make(0, i))) cand.push_back(i);
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
    tune_cache_put(pb, best_i, best);
    return ICL_OK;
}

icl_status tune_conv(const Problem& pb, hipStream_t st) {
    const icl_op op = pb.op;
    const icl_dtype dt = pb.dt;
    const int r = pb.r, W = pb.W, H = pb.H;
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
        return search(pb, tab, count, sets, make, agree, st);
    } else {
        int count;
        const Variant<Conv2dArgs>* tab = conv2d_variants(&count);
        auto make = [&](int s, int) { return Conv2dArgs{src[s], pitch, dst[s], pitch, W, H, dt, d_taps, r, st}; };
        Conv2dArgs p0 = make(0, 0);
        p0.dst = ref;
        if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
        auto agree = [&]() { return outputs_agree(dt, dst[0], ref, pitch, W, H, d_stat, st); };
        return search(pb, tab, count, sets, make, agree, st);
    }
}

icl_status tune_harris(const Problem& pb, hipStream_t st) {
    const int rg = pb.r, W = pb.W, H = pb.H;
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
    // the response cancels (det - k tr^2), so it is compared against its largest magnitude
    auto agree = [&]() { return outputs_agree(ICL_F32, dst[0], ref, pitch, W, H, d_stat, st, Agree::Max); };
    return search(pb, tab, count, sets, make, agree, st);
}

icl_status tune_conv_u8(const Problem& pb, hipStream_t st) {
    const int r = pb.r, W = pb.W, H = pb.H;
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
    return search(pb, tab, count, sets, make, agree, st);
}

// Fused corners: the single-pass variants share their arithmetic, so each must return the
// default single-pass variant's mask byte for byte (the two-kernel variant is not a candidate).
icl_status tune_corners(const Problem& pb, hipStream_t st) {
    const int rg = pb.r, W = pb.W, H = pb.H;
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
    return search(pb, tab, count, sets, make, agree, st);
}

icl_status tune_nms(const Problem& pb, hipStream_t st) {
    const int r = pb.r, W = pb.W, H = pb.H;
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
    return search(pb, tab, count, sets, make, agree, st);
}

// Separable 3-D correlation: volumes of W x H x D voxels whose slices follow each other
// (slice pitch = H row pitches), so the whole volume reads as one W x (H D) image for
// filling and comparing.
icl_status tune_sep3d(const Problem& pb, hipStream_t st) {
    const icl_dtype dt = pb.dt;
    const int r = pb.r, W = pb.W, H = pb.H, D = pb.D;
    const int es = elem_size(dt);
    const size_t pitch = ((size_t)W * es + 255) & ~(size_t)255, spitch = pitch * H, bytes = spitch * D;
    if ((size_t)H * D > (size_t)INT32_MAX) return ICL_ERR_UNSUPPORTED;
    const int HD = H * D;
    const int sets = rotation_sets(2 * bytes);
    Buffers b;
    std::vector<void*> src(sets), dst(sets);
    for (int s = 0; s < sets; ++s) {
        src[s] = b.alloc(bytes);
        dst[s] = b.alloc(bytes);
        if (!src[s] || !dst[s]) return ICL_ERR_HIP;
        if (fill(dt, src[s], pitch, W, HD, 0x3d3dull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(bytes);
    const int n = 2 * r + 1;
    std::vector<float> taps(3 * n);
    for (int a = 0; a < 3; ++a) {
        double sum = 0;
        for (int k = 0; k < n; ++k) sum += (taps[a * n + k] = 1.0f + 0.25f * (float)(((k + a) * 7) % 5));
        for (int k = 0; k < n; ++k) taps[a * n + k] = (float)(taps[a * n + k] / sum);
    }
    float* d_taps = static_cast<float*>(b.alloc(taps.size() * sizeof(float)));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    const size_t wsb = sep3d_workspace(W, H, D);
    void* ws = b.alloc(wsb);
    if (!ref || !d_taps || !d_stat || !ws) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_taps, taps.data(), taps.size() * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
        return ICL_ERR_HIP;
    int count;
    const Variant<Sep3Args>* tab = sep3d_variants(&count);
    auto make = [&](int s, int) {
        return Sep3Args{src[s], pitch, spitch, dst[s], pitch, spitch, W, H, D, dt, d_taps, d_taps + n, d_taps + 2 * n,
                        r, ws, wsb, st};
    };
    Sep3Args p0 = make(0, 0);
    p0.dst = ref;
    if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    auto agree = [&]() { return outputs_agree(dt, dst[0], ref, pitch, W, HD, d_stat, st); };
    return search(pb, tab, count, sets, make, agree, st);
}

// Filter bank (forward, input adjoint, filter adjoint): x [N][H][W], w [F][k][k], y or gy
// [N][F][H][W], on positive inputs and positive normalised taps so that every output is a
// sum of non-negative terms and the per-element comparison is the normwise one.
icl_status tune_bank(const Problem& pb, hipStream_t st) {
    const icl_op op = pb.op;
    const int r = pb.r, W = pb.W, H = pb.H, N = pb.N, F = pb.F;
    const size_t hw = (size_t)H * W, nk = (size_t)(2 * r + 1) * (2 * r + 1);
    const size_t xb = (size_t)N * hw * 4, yb = (size_t)N * F * hw * 4, wb = (size_t)F * nk * 4;
    if ((size_t)N * F * H > (size_t)INT32_MAX) return ICL_ERR_UNSUPPORTED;
    // the operation's input and output
    const size_t inb = op == ICL_OP_BANK_BWD_INPUT ? yb : xb;
    const size_t outb = op == ICL_OP_BANK_FWD ? yb : (op == ICL_OP_BANK_BWD_INPUT ? xb : wb);
    const size_t sideb = op == ICL_OP_BANK_BWD_FILTER ? yb : 0;   // gy beside x for the filter adjoint
    const int sets = rotation_sets(inb + outb + sideb);
    Buffers b;
    std::vector<void*> in(sets), out(sets), side(sets);
    for (int s = 0; s < sets; ++s) {
        in[s] = b.alloc(inb);
        out[s] = b.alloc(outb);
        side[s] = sideb ? b.alloc(sideb) : nullptr;
        if (!in[s] || !out[s] || (sideb && !side[s])) return ICL_ERR_HIP;
        if (fill(ICL_F32, in[s], (size_t)W * 4, W, (int)(inb / 4 / W), 0xb0ull + s, st) != hipSuccess) return ICL_ERR_HIP;
        if (sideb && fill(ICL_F32, side[s], (size_t)W * 4, W, (int)(sideb / 4 / W), 0xc0ull + s, st) != hipSuccess)
            return ICL_ERR_HIP;
    }
    void* ref = b.alloc(outb);
    std::vector<float> w(F * nk);
    for (int f = 0; f < F; ++f) {
        double sum = 0;
        for (size_t k = 0; k < nk; ++k) sum += (w[f * nk + k] = 1.0f + 0.25f * (float)((k * 7 + f) % 5));
        for (size_t k = 0; k < nk; ++k) w[f * nk + k] = (float)(w[f * nk + k] / sum);
    }
    float* d_w = static_cast<float*>(b.alloc(wb));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    const size_t wsb = op == ICL_OP_BANK_BWD_FILTER ? bank_bwd_filter_workspace(N, F, H, W, r) : 0;
    void* ws = wsb ? b.alloc(wsb) : nullptr;
    if (!ref || !d_w || !d_stat || (wsb && !ws)) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_w, w.data(), wb, hipMemcpyHostToDevice, st) != hipSuccess) return ICL_ERR_HIP;
    int count;
    const Variant<BankArgs>* tab = op == ICL_OP_BANK_FWD ? bank_fwd_variants(&count)
                                   : op == ICL_OP_BANK_BWD_INPUT ? bank_bwd_input_variants(&count)
                                                                 : bank_bwd_filter_variants(&count);
    auto make = [&](int s, int) {
        if (op == ICL_OP_BANK_BWD_FILTER)   // a = gy, b = x
            return BankArgs{static_cast<const float*>(side[s]), static_cast<const float*>(in[s]),
                            static_cast<float*>(out[s]), N, F, H, W, r, ws, wsb, st};
        return BankArgs{static_cast<const float*>(in[s]), d_w, static_cast<float*>(out[s]), N, F, H, W, r, nullptr, 0,
                        st};
    };
    BankArgs p0 = make(0, 0);
    p0.out = static_cast<float*>(ref);
    if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    // output viewed as an image of W-wide rows (the filter gradient as one row of F k^2 values)
    const int ow = op == ICL_OP_BANK_BWD_FILTER ? (int)(F * nk) : W;
    const int oh = (int)(outb / 4 / ow);
    // the filter gradient reduces N H W terms per tap in blocks: a looser bound than one stencil
    const float tol = op == ICL_OP_BANK_BWD_FILTER ? 1e-4f : 1e-5f;
    auto agree = [&]() {
        return outputs_agree(ICL_F32, out[0], ref, (size_t)ow * 4, ow, oh, d_stat, st, Agree::PerPixel, tol);
    };
    return search(pb, tab, count, sets, make, agree, st);
}

// Filter-bank forward fused with the loss: candidates must reproduce the reference
// variant's gradient gy = 2 (y - t) (relative to its largest magnitude: gy changes sign)
// and its loss.
icl_status tune_bank_sse(const Problem& pb, hipStream_t st) {
    const int r = pb.r, W = pb.W, H = pb.H, N = pb.N, F = pb.F;
    const size_t hw = (size_t)H * W, nk = (size_t)(2 * r + 1) * (2 * r + 1);
    const size_t xb = (size_t)N * hw * 4, yb = (size_t)N * F * hw * 4, wb = (size_t)F * nk * 4;
    if ((size_t)N * F * H > (size_t)INT32_MAX) return ICL_ERR_UNSUPPORTED;
    const int sets = rotation_sets(xb + 2 * yb);
    Buffers b;
    std::vector<void*> x(sets), t(sets), gy(sets);
    for (int s = 0; s < sets; ++s) {
        x[s] = b.alloc(xb);
        t[s] = b.alloc(yb);
        gy[s] = b.alloc(yb);
        if (!x[s] || !t[s] || !gy[s]) return ICL_ERR_HIP;
        if (fill(ICL_F32, x[s], (size_t)W * 4, W, N * H, 0xd0ull + s, st) != hipSuccess) return ICL_ERR_HIP;
        if (fill(ICL_F32, t[s], (size_t)W * 4, W, N * F * H, 0xe0ull + s, st) != hipSuccess) return ICL_ERR_HIP;
    }
    void* ref = b.alloc(yb);
    std::vector<float> w(F * nk);
    for (int f = 0; f < F; ++f) {
        double sum = 0;
        for (size_t k = 0; k < nk; ++k) sum += (w[f * nk + k] = 1.0f + 0.25f * (float)((k * 7 + f) % 5));
        for (size_t k = 0; k < nk; ++k) w[f * nk + k] = (float)(w[f * nk + k] / sum);
    }
    float* d_w = static_cast<float*>(b.alloc(wb));
    unsigned* d_stat = static_cast<unsigned*>(b.alloc(16));
    float* d_loss = static_cast<float*>(b.alloc(16));
    const size_t wsb = bank_fwd_sse_workspace();
    void* ws = b.alloc(wsb);
    if (!ref || !d_w || !d_stat || !d_loss || !ws) return ICL_ERR_HIP;
    if (hipMemcpyAsync(d_w, w.data(), wb, hipMemcpyHostToDevice, st) != hipSuccess) return ICL_ERR_HIP;
    int count;
    const Variant<BankSseArgs>* tab = bank_fwd_sse_variants(&count);
    auto make = [&](int s, int) {
        return BankSseArgs{static_cast<const float*>(x[s]), d_w, static_cast<const float*>(t[s]), nullptr,
                           static_cast<float*>(gy[s]), d_loss, N, F, H, W, r, ws, wsb, st};
    };
    BankSseArgs p0 = make(0, 0);
    p0.gy = static_cast<float*>(ref);
    if (!tab[0].supports(p0) || tab[0].launch(p0) != hipSuccess) return ICL_ERR_HIP;
    float ref_loss = 0.f;
    if (hipMemcpyAsync(&ref_loss, d_loss, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return ICL_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return ICL_ERR_HIP;
    auto agree = [&]() {
        float l = 0.f;
        if (hipMemcpyAsync(&l, d_loss, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        if (hipStreamSynchronize(st) != hipSuccess) return false;
        if (!(std::fabs(l - ref_loss) <= 1e-5f * std::fabs(ref_loss))) return false;
        return outputs_agree(ICL_F32, gy[0], ref, (size_t)W * 4, W, N * F * H, d_stat, st, Agree::Max, 1e-5f);
    };
    return search(pb, tab, count, sets, make, agree, st);
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

void tune_cache_put(const Problem& p, int variant, double us) {
    const char* name = icl_variant_name(p.op, variant);
    if (!name) return;
    const std::string key = make_key(p);
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = Entry{name, us};
}

int tune_cache_get(const Problem& p) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_cache.empty()) return -1;
    }
    const std::string key = make_key(p);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return -1;
    return index_of(p.op, it->second.variant);
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
    const icl_problem q{op, dtype, radius, width, height, 1, 1, 1};
    return icl_tune_problem(&q, stream);
}

icl_status icl_tune_problem(const icl_problem* q, void* stream) {
    if (!q) return ICL_ERR_INVALID_VALUE;
    const Problem pb = problem_of(*q);
    const icl_op op = pb.op;
    const icl_dtype dtype = pb.dt;
    const int radius = pb.r;
    if (pb.W < 1 || pb.H < 1 || q->depth < 0 || q->n < 0 || q->f < 0) return ICL_ERR_INVALID_VALUE;
    if (op == ICL_OP_CONV_SEP_BATCHED) return ICL_ERR_INVALID_VALUE;   // tuned per plan: icl_batch_plan_tune
    if (op == ICL_OP_CONV2D_U8 ? dtype != ICL_U8 : (dtype != ICL_F32 && dtype != ICL_F16 && dtype != ICL_BF16))
        return ICL_ERR_DTYPE;
    // every argument is checked before the device is touched
    switch (op) {
        case ICL_OP_CONV_SEP: case ICL_OP_CONV2D:
            if (radius < 0 || radius > ICL_MAX_RADIUS) return ICL_ERR_RADIUS;
            break;
        case ICL_OP_HARRIS: case ICL_OP_CORNERS:
            if (radius < 0 || radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            break;
        case ICL_OP_NMS:
            if (radius < 1 || radius > ICL_MAX_NMS_RADIUS) return ICL_ERR_RADIUS;
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            break;
        case ICL_OP_CONV2D_U8:
            if (radius < 0 || radius > ICL_MAX_U8_RADIUS) return ICL_ERR_RADIUS;
            break;
        case ICL_OP_CONV3D_SEP:
            if (radius < 0 || radius > ICL_MAX_RADIUS_3D) return ICL_ERR_RADIUS;
            break;
        case ICL_OP_BANK_FWD: case ICL_OP_BANK_BWD_INPUT: case ICL_OP_BANK_BWD_FILTER: case ICL_OP_BANK_FWD_SSE:
            if (dtype != ICL_F32) return ICL_ERR_DTYPE;
            if (radius < 1 || radius > 4) return ICL_ERR_RADIUS;
            if (pb.F > 64) return ICL_ERR_UNSUPPORTED;
            break;
        case ICL_OP_SSE_LOSS: break;
        default: return ICL_ERR_INVALID_VALUE;
    }
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ICL_ERR_UNSUPPORTED;
    switch (op) {
        case ICL_OP_CONV_SEP:
        case ICL_OP_CONV2D:
            s = tune_conv(pb, st);
            break;
        case ICL_OP_HARRIS:
            s = tune_harris(pb, st);
            break;
        case ICL_OP_CORNERS:
            if (radius > 3) return ICL_OK;   // only the two-kernel variant runs such windows: nothing to choose
            s = tune_corners(pb, st);
            break;
        case ICL_OP_CONV2D_U8:
            s = tune_conv_u8(pb, st);
            break;
        case ICL_OP_NMS:
            s = tune_nms(pb, st);
            break;
        case ICL_OP_CONV3D_SEP:
            s = tune_sep3d(pb, st);
            break;
        case ICL_OP_BANK_FWD: case ICL_OP_BANK_BWD_INPUT: case ICL_OP_BANK_BWD_FILTER:
            s = tune_bank(pb, st);
            break;
        case ICL_OP_BANK_FWD_SSE:
            s = tune_bank_sse(pb, st);
            break;
        case ICL_OP_SSE_LOSS:
            return ICL_OK;   // one variant (the fixed-order two-stage reduction): nothing to choose
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
