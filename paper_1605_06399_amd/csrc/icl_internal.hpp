// Host-side internals: argument bundles, the variant registry and helpers
// shared by the entry points, the kernels' launchers and the tuner.
#pragma once
#include <hip/hip_runtime.h>

#include "icl_device.hpp"
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/icl.h"

namespace icl {

inline int elem_size(icl_dtype d) { return d == ICL_F32 ? 4 : (d == ICL_U8 ? 1 : 2); }

struct SepArgs {
    const void* src; size_t sp; void* dst; size_t dp;
    int W, H; icl_dtype dt;
    const float* tx; const float* ty; int r;
    void* ws; size_t wsb;
    hipStream_t st;
    Border bd{};
};

struct Conv2dArgs {
    const void* src; size_t sp; void* dst; size_t dp;
    int W, H; icl_dtype dt;
    const float* taps; int r;
    hipStream_t st;
    Border bd{};
};

struct U8Args {
    const uint8_t* src; size_t sp; uint8_t* dst; size_t dp;
    int W, H;
    const int16_t* taps; int r; int shift;
    int cmode; int cval;   // constant boundary flag and its value (0..255)
    hipStream_t st;
};

struct Sep3Args {
    const void* src; size_t srp, ssp;   // row and slice pitches (bytes)
    void* dst; size_t drp, dsp;
    int W, H, D; icl_dtype dt;
    const float *tx, *ty, *tz; int r;
    void* ws; size_t wsb;
    hipStream_t st;
    Border bd{};
};

struct HarrisArgs {
    const float* src; size_t sp; float* resp; size_t rp;
    int W, H;
    const float* g; int rg; float k;
    void* ws; size_t wsb;
    hipStream_t st;
};

struct NmsArgs {
    const float* R; size_t rp; uint8_t* M; size_t mp;
    int W, H; int r; float tau;
    hipStream_t st;
};

struct CornersArgs {
    const float* src; size_t sp; uint8_t* M; size_t mp;
    int W, H;
    const float* g; int rg; float k;   // Harris window taps, radius, k
    int nr; float tau;                 // NMS radius and threshold
    float* resp; size_t rp;            // optional response output (null: not written)
    void* ws; size_t wsb;
    hipStream_t st;
};

struct BankArgs {
    const float* a;   // x (fwd, bwd_filter) or gy (bwd_input)
    const float* b;   // w (fwd, bwd_input) or x (bwd_filter: a = gy, b = x)
    float* out;
    int n, f, h, w, r;
    void* ws; size_t wsb;
    hipStream_t st;
    const float* scale = nullptr;   // adjoints: device factor on the output (null = 1)
};

struct BankSseArgs {
    const float *x, *w, *t;
    float *y, *gy, *loss;   // y and gy may be null
    int n, f, h, wd, r;
    void* ws; size_t wsb;
    hipStream_t st;
};

// One precompiled candidate implementation of an operation.
template <class A> struct Variant {
    const char* name;
    bool (*supports)(const A&);        // can this variant run these arguments?
    hipError_t (*launch)(const A&);
};

// Small neural-network time model of the model-guided tuner (host code).
struct PerfModel {
    int d = 0, h = 0;
    std::vector<double> mu, sd, p;
    double ymu = 0.0, ysd = 1.0;
    bool fit(const std::vector<std::vector<double>>& X, const std::vector<double>& y, int hidden, int iters,
             uint64_t seed);
    double predict(const std::vector<double>& x) const;
};
// Feature vectors of variants from their names (family one-hot, log2 of numeric parameters).
void variant_features(const std::vector<std::string>& names, std::vector<std::vector<double>>& F);

// Variant tables (index 0 = plain one-pixel-per-thread kernel).
const Variant<SepArgs>* sep_variants(int* count);
const Variant<Conv2dArgs>* conv2d_variants(int* count);
const Variant<U8Args>* conv2d_u8_variants(int* count);
const Variant<HarrisArgs>* harris_variants(int* count);
const Variant<NmsArgs>* nms_variants(int* count);
const Variant<CornersArgs>* corners_variants(int* count);
const Variant<Sep3Args>* sep3d_variants(int* count);
const Variant<BankArgs>* bank_fwd_variants(int* count);
const Variant<BankArgs>* bank_bwd_input_variants(int* count);
const Variant<BankArgs>* bank_bwd_filter_variants(int* count);
const Variant<BankSseArgs>* bank_fwd_sse_variants(int* count);

// Default choice when neither a forced variant nor a tune-cache entry applies.
int sep_default(const SepArgs&);
int conv2d_default(const Conv2dArgs&);
bool supports_conv2d_mfma(const Conv2dArgs&);       // the matrix-core variant (conv2d_mfma.hip)
hipError_t launch_conv2d_mfma(const Conv2dArgs&);
int conv2d_u8_default(const U8Args&);
int harris_default(const HarrisArgs&);
int nms_default(const NmsArgs&);
int corners_default(const CornersArgs&);
int sep3d_default(const Sep3Args&);
int bank_fwd_default(const BankArgs&);
int bank_bwd_input_default(const BankArgs&);
int bank_bwd_filter_default(const BankArgs&);
int bank_fwd_sse_default(const BankSseArgs&);
int batched_default();

size_t sep_workspace(int W, int H);
size_t harris_workspace(int W, int H);
size_t corners_workspace(int W, int H, int rg);
size_t sep3d_workspace(int W, int H, int D);
size_t bank_bwd_filter_workspace(int n, int f, int h, int w, int r);
size_t sse_workspace(long long count);
size_t bank_fwd_sse_workspace();
// Most work-groups of a fused forward + loss launch: one float64 loss partial each in the
// workspace, so the workspace is the same for every problem size.
constexpr int FWD_SSE_PARTS = 2048;

hipError_t sse_launch(const float* y, const float* t, float* gy, long long count, float* loss,
                      void* ws, size_t wsb, hipStream_t st);


// A problem as the tuner keys it: the operation, storage type, radius and the sizes that
// change which variant is fastest (depth of a volume, batch and filter counts of the bank).
struct Problem {
    icl_op op;
    icl_dtype dt;
    int r;
    int W, H;
    int D = 1, N = 1, F = 1;
};
inline Problem problem_of(const icl_problem& p) {
    return Problem{p.op, p.dtype, p.radius, p.width, p.height, p.depth > 1 ? p.depth : 1, p.n > 1 ? p.n : 1,
                   p.f > 1 ? p.f : 1};
}

// Variant selection shared by the entry points: forced > tune cache > default.  With
// ICL_TUNE=search and a stream, a cache miss is tuned first (outside stream capture).
int select_variant(const Problem& p, int fallback, hipStream_t st = nullptr);
inline int select_variant(icl_op op, icl_dtype dt, int r, int W, int H, int fallback, hipStream_t st = nullptr) {
    return select_variant(Problem{op, dt, r, W, H}, fallback, st);
}
bool variant_forced(icl_op op);
// Whether the process-wide arithmetic mode (icl_set_math) lets tuning and default
// selection pick this variant.
bool variant_allowed(icl_op op, int index);
int math_mode();

// Tuner hooks (tuner.hip).
void tune_cache_put(const Problem& p, int variant, double us);
int tune_cache_get(const Problem& p);
// Plan-level search of the batched walks (batched.hip); caches the winner for the plan.
icl_status tune_batch_plan(icl_batch_plan* plan, hipStream_t st);

// Lazily checks that a HIP device is visible (ICL_ERR_NO_DEVICE otherwise).
icl_status device_ready();
const char* op_name(icl_op op);

// Grid for a persistent tile loop: resident blocks of `kernel` on the whole device
// (occupancy x CUs, cached per kernel), at most `ntiles`, rounded down to a multiple of 8.
int persistent_grid(const void* kernel, int block, int ntiles);

// Zero-fill `n` floats with a kernel (no memset node, so it is safe inside captured graphs).
hipError_t zero_fill(float* p, size_t n, hipStream_t st);

// Thread-local HIP error bookkeeping.
void set_hip_error(hipError_t e);
inline icl_status hip_status(hipError_t e) {
    if (e == hipSuccess) return ICL_OK;
    set_hip_error(e);
    return ICL_ERR_HIP;
}

}  // namespace icl
