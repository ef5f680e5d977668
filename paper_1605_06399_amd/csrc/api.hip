// C-ABI entry points: argument validation on the host, variant selection and
// launch.  The standalone host function of the paper's code generator
// (Section 5.1) is the model: one call per stencil, plain pointers and sizes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "icl_internal.hpp"

using namespace icl;

namespace icl {

static thread_local int g_last_hip_error = 0;
static void* scratch_on_current_device();
void set_hip_error(hipError_t e) { g_last_hip_error = (int)e; }

static std::atomic<int> g_forced[ICL_OP_COUNT] = {};
static std::once_flag g_force_env_once;
static int g_device_state = -1;     // -1 unknown, 0 none, 1 ok
static std::mutex g_init_mu;

static const char* kOpNames[ICL_OP_COUNT] = {"conv_sep", "conv2d", "harris", "nms", "conv_sep_batched",
                                             "bank_fwd", "bank_bwd_input", "bank_bwd_filter", "sse_loss",
                                             "bank_fwd_sse", "conv2d_u8", "corners", "conv3d_sep"};

// ICL_FORCE_VARIANT="conv_sep=1,conv2d=3": the analogue of the paper's directives
// that force optimisations on or off.
static void parse_force_env() {
    for (int i = 0; i < ICL_OP_COUNT; ++i) g_forced[i] = -1;
    const char* e = std::getenv("ICL_FORCE_VARIANT");
    if (!e) return;
    std::string s(e);
    size_t pos = 0;
    while (pos < s.size()) {
        size_t end = s.find(',', pos);
        if (end == std::string::npos) end = s.size();
        const std::string item = s.substr(pos, end - pos);
        const size_t eq = item.find('=');
        if (eq != std::string::npos) {
            const std::string name = item.substr(0, eq);
            const int idx = std::atoi(item.c_str() + eq + 1);
            for (int i = 0; i < ICL_OP_COUNT; ++i)
                if (name == kOpNames[i]) g_forced[i] = idx;
        }
        pos = end + 1;
    }
}

static void ensure_force_env() { std::call_once(g_force_env_once, parse_force_env); }

bool variant_forced(icl_op op) {
    ensure_force_env();
    return g_forced[op].load() >= 0;
}

static std::atomic<int> g_math{ICL_MATH_F32};
int math_mode() { return g_math.load(); }

static const char* arith_of(icl_op op, const char* name) {
    if (!name) return nullptr;
    if (op == ICL_OP_CONV2D_U8) return "int32_valu";
    if (std::strncmp(name, "mfma_f16", 8) == 0) return "fp16x3_mfma";
    if (std::strstr(name, "mfma")) return "fp32_mfma";
    return "fp32_valu";
}

bool variant_allowed(icl_op op, int index) {
    const char* a = arith_of(op, icl_variant_name(op, index));
    if (!a) return false;
    return std::strcmp(a, "fp16x3_mfma") != 0 || g_math.load() == ICL_MATH_F16_SPLIT;
}

// ICL_TUNE: 0 off (cache ignored), 1 cache (default), 2 search on a miss
static int g_tune_mode = 1;
static std::string g_tune_file;
static std::once_flag g_tune_env_once;

static void parse_tune_env() {
    if (const char* e = std::getenv("ICL_TUNE")) {
        const std::string v(e);
        if (v == "off") g_tune_mode = 0;
        else if (v == "search") g_tune_mode = 2;
        else g_tune_mode = 1;
    }
    if (const char* f = std::getenv("ICL_TUNE_CACHE")) {
        g_tune_file = f;
        if (g_tune_mode > 0) icl_tune_load(f);   // a missing or foreign file leaves the cache empty
    }
}

static bool tunable(icl_op op) {
    switch (op) {
        case ICL_OP_CONV_SEP: case ICL_OP_CONV2D: case ICL_OP_HARRIS: case ICL_OP_NMS: case ICL_OP_CONV2D_U8:
        case ICL_OP_CORNERS: case ICL_OP_CONV3D_SEP: case ICL_OP_BANK_FWD: case ICL_OP_BANK_BWD_INPUT:
        case ICL_OP_BANK_BWD_FILTER: case ICL_OP_BANK_FWD_SSE: return true;
        default: return false;
    }
}

int select_variant(const Problem& p, int fallback, hipStream_t st) {
    ensure_force_env();
    std::call_once(g_tune_env_once, parse_tune_env);
    const int f = g_forced[p.op].load();
    if (f >= 0) return f;
    if (g_tune_mode == 0) return fallback;
    int c = tune_cache_get(p);
    if (c < 0 && g_tune_mode == 2 && st != nullptr && tunable(p.op)) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const icl_problem q{p.op, p.dt, p.r, p.W, p.H, p.D, p.N, p.F};
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
            icl_tune_problem(&q, st) == ICL_OK) {
            icl_tune_save(g_tune_file.empty() ? nullptr : g_tune_file.c_str());
            c = tune_cache_get(p);
        }
    }
    if (c >= 0 && variant_allowed(p.op, c)) return c;
    return fallback;
}

const char* op_name(icl_op op) { return (op >= 0 && op < ICL_OP_COUNT) ? kOpNames[op] : "?"; }

icl_status device_ready() {
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_device_state < 0) {
        int n = 0;
        const hipError_t e = hipGetDeviceCount(&n);
        g_device_state = (e == hipSuccess && n > 0) ? 1 : 0;
    }
    return g_device_state == 1 ? ICL_OK : ICL_ERR_NO_DEVICE;
}

static std::mutex g_occ_mu;
static std::vector<std::pair<const void*, int>> g_occ;   // kernel -> resident blocks on the device
static int g_cus = 0;

int persistent_grid(const void* kernel, int block, int ntiles) {
    int resident = 0;
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        for (const auto& e : g_occ)
            if (e.first == kernel) resident = e.second;
        if (resident == 0) {
            if (g_cus == 0) {
                int dev = 0;
                if (hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                    g_cus = 1;
            }
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            resident = per_cu * g_cus;
            g_occ.push_back({kernel, resident});
        }
    }
    int g = ntiles < resident ? ntiles : resident;
    if (g > 8) g -= g % 8;
    return g < 1 ? 1 : g;
}

}  // namespace icl

namespace {

bool dtype_ok(icl_dtype d) { return d == ICL_F32 || d == ICL_F16 || d == ICL_BF16; }

icl::Border border_of(icl_border b, float value) {
    icl::Border bd;
    bd.constant = b == ICL_BORDER_CONSTANT ? 1 : 0;
    bd.value = bd.constant ? value : 0.f;
    return bd;
}

// Image checks shared by the entry points (sizes already known to be >= 1).
icl_status check_image(const void* p, size_t pitch, int W, int es) {
    if (!p) return ICL_ERR_INVALID_VALUE;
    if (pitch < (size_t)W * (size_t)es || pitch % (size_t)es) return ICL_ERR_PITCH;
    return ICL_OK;
}

// Byte ranges [p, p + (H-1)*pitch + W*es) of two images intersect.
bool overlaps(const void* a, size_t ap, int aes, const void* b, size_t bp, int bes, int W, int H) {
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (size_t)(H - 1) * ap + (size_t)W * aes;
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + (size_t)(H - 1) * bp + (size_t)W * bes;
    return a0 < b1 && b0 < a1;
}

bool range_overlaps(const void* a, size_t an, const void* b, size_t bn) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bn && b0 < a0 + an;
}

// Run the chosen variant; fall back to the default (or plain) when a tuned choice
// cannot run these arguments.  Forced choices never fall back.
template <class A>
icl_status dispatch(icl_op op, const Variant<A>* tab, int count, const A& a, int chosen, int deflt) {
    const bool forced = variant_forced(op);
    if (chosen < 0 || chosen >= count) {
        if (forced) return ICL_ERR_UNSUPPORTED;
        chosen = deflt;
    }
    if (!tab[chosen].supports(a)) {
        if (forced) return ICL_ERR_UNSUPPORTED;
        chosen = deflt;
        if (!tab[chosen].supports(a)) {
            chosen = 0;
            if (!tab[0].supports(a)) return ICL_ERR_UNSUPPORTED;
        }
    }
    return hip_status(tab[chosen].launch(a));
}

}  // namespace

extern "C" {

icl_status icl_init(void) {
    const icl_status s = device_ready();
    if (s != ICL_OK) return s;
    return scratch_on_current_device() ? ICL_OK : ICL_ERR_HIP;
}

const char* icl_version(void) { return "icl 0.1 (gfx950)"; }

int icl_last_hip_error(void) { return g_last_hip_error; }

const char* icl_status_string(icl_status s) {
    switch (s) {
        case ICL_OK: return "ok";
        case ICL_ERR_INVALID_VALUE: return "invalid value";
        case ICL_ERR_PITCH: return "invalid pitch";
        case ICL_ERR_RADIUS: return "radius out of range";
        case ICL_ERR_DTYPE: return "unsupported storage type";
        case ICL_ERR_ALIAS: return "output overlaps an input";
        case ICL_ERR_WORKSPACE: return "workspace missing or too small";
        case ICL_ERR_NO_DEVICE: return "no HIP device";
        case ICL_ERR_HIP: return "HIP runtime error";
        case ICL_ERR_UNSUPPORTED: return "unsupported request";
        case ICL_ERR_TUNE_CACHE: return "tune cache unreadable or foreign";
    }
    return "unknown status";
}

icl_status icl_workspace_size(icl_op op, int width, int height, int n, int f, int radius, icl_dtype dtype,
                              size_t* bytes) {
    if (!bytes) return ICL_ERR_INVALID_VALUE;
    if (width < 0 || height < 0 || n < 0 || f < 0) return ICL_ERR_INVALID_VALUE;
    if (op == ICL_OP_CONV2D_U8 ? dtype != ICL_U8 : !dtype_ok(dtype)) return ICL_ERR_DTYPE;
    *bytes = 0;
    switch (op) {
        case ICL_OP_CONV_SEP: *bytes = sep_workspace(width, height); break;
        case ICL_OP_HARRIS: *bytes = harris_workspace(width, height); break;
        case ICL_OP_BANK_BWD_FILTER:
            if (radius < 1 || radius > 4) return ICL_ERR_RADIUS;
            *bytes = bank_bwd_filter_workspace(n, f, height, width, radius);
            break;
        case ICL_OP_SSE_LOSS: *bytes = sse_workspace((long long)width * height); break;
        case ICL_OP_BANK_FWD_SSE: *bytes = bank_fwd_sse_workspace(); break;
        case ICL_OP_CORNERS:
            if (radius < 0 || radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
            *bytes = corners_workspace(width, height, radius);
            break;
        case ICL_OP_CONV3D_SEP: *bytes = sep3d_workspace(width, height, n); break;
        case ICL_OP_CONV2D: case ICL_OP_NMS: case ICL_OP_CONV_SEP_BATCHED: case ICL_OP_BANK_FWD:
        case ICL_OP_BANK_BWD_INPUT: case ICL_OP_CONV2D_U8: break;
        default: return ICL_ERR_INVALID_VALUE;
    }
    return ICL_OK;
}

icl_status icl_conv_sep(const void* src, size_t src_pitch, void* dst, size_t dst_pitch, int width, int height,
                        icl_dtype dtype, const float* taps_x, const float* taps_y, int radius, void* workspace,
                        size_t workspace_bytes, void* stream) {
    return icl_conv_sep_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius,
                               ICL_BORDER_CLAMP, 0.f, workspace, workspace_bytes, stream);
}

icl_status icl_conv_sep_border(const void* src, size_t src_pitch, void* dst, size_t dst_pitch, int width,
                               int height, icl_dtype dtype, const float* taps_x, const float* taps_y, int radius,
                               icl_border border, float constant, void* workspace, size_t workspace_bytes,
                               void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (border != ICL_BORDER_CLAMP && border != ICL_BORDER_CONSTANT) return ICL_ERR_INVALID_VALUE;
    if (!dtype_ok(dtype)) return ICL_ERR_DTYPE;
    if (radius < 0 || radius > ICL_MAX_RADIUS) return ICL_ERR_RADIUS;
    if (width == 0 || height == 0) return ICL_OK;
    const int es = elem_size(dtype);
    icl_status s;
    if ((s = check_image(src, src_pitch, width, es)) != ICL_OK) return s;
    if ((s = check_image(dst, dst_pitch, width, es)) != ICL_OK) return s;
    if (!taps_x || !taps_y) return ICL_ERR_INVALID_VALUE;
    if (overlaps(src, src_pitch, es, dst, dst_pitch, es, width, height)) return ICL_ERR_ALIAS;
    if (workspace && (range_overlaps(workspace, workspace_bytes, dst,
                                     (size_t)(height - 1) * dst_pitch + (size_t)width * es) ||
                      range_overlaps(workspace, workspace_bytes, src,
                                     (size_t)(height - 1) * src_pitch + (size_t)width * es)))
        return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    SepArgs a{src, src_pitch, dst, dst_pitch, width, height, dtype, taps_x, taps_y, radius,
              workspace, workspace_bytes, (hipStream_t)stream, border_of(border, constant)};
    int count;
    const Variant<SepArgs>* tab = sep_variants(&count);
    const int deflt = sep_default(a);
    const int v = select_variant(ICL_OP_CONV_SEP, dtype, radius, width, height, deflt, a.st);
    // the two-pass variants (and every radius above the fused kernels' range) need the intermediate
    const bool forced_two_pass = variant_forced(ICL_OP_CONV_SEP) && v == 0;
    if ((forced_two_pass || !tab[deflt].supports(a)) && !tab[0].supports(a)) return ICL_ERR_WORKSPACE;
    return dispatch(ICL_OP_CONV_SEP, tab, count, a, v, deflt);
}

icl_status icl_conv2d(const void* src, size_t src_pitch, void* dst, size_t dst_pitch, int width, int height,
                      icl_dtype dtype, const float* taps, int radius, void* stream) {
    return icl_conv2d_border(src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, ICL_BORDER_CLAMP,
                             0.f, stream);
}

icl_status icl_conv2d_border(const void* src, size_t src_pitch, void* dst, size_t dst_pitch, int width, int height,
                             icl_dtype dtype, const float* taps, int radius, icl_border border, float constant,
                             void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (border != ICL_BORDER_CLAMP && border != ICL_BORDER_CONSTANT) return ICL_ERR_INVALID_VALUE;
    if (!dtype_ok(dtype)) return ICL_ERR_DTYPE;
    if (radius < 0 || radius > ICL_MAX_RADIUS) return ICL_ERR_RADIUS;
    if (width == 0 || height == 0) return ICL_OK;
    const int es = elem_size(dtype);
    icl_status s;
    if ((s = check_image(src, src_pitch, width, es)) != ICL_OK) return s;
    if ((s = check_image(dst, dst_pitch, width, es)) != ICL_OK) return s;
    if (!taps) return ICL_ERR_INVALID_VALUE;
    if (overlaps(src, src_pitch, es, dst, dst_pitch, es, width, height)) return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    Conv2dArgs a{src, src_pitch, dst, dst_pitch, width, height, dtype, taps, radius, (hipStream_t)stream,
                 border_of(border, constant)};
    int count;
    const Variant<Conv2dArgs>* tab = conv2d_variants(&count);
    const int deflt = conv2d_default(a);
    return dispatch(ICL_OP_CONV2D, tab, count, a, select_variant(ICL_OP_CONV2D, dtype, radius, width, height, deflt, a.st),
                    deflt);
}

icl_status icl_conv3d_sep(const void* src, size_t src_row_pitch, size_t src_slice_pitch, void* dst,
                          size_t dst_row_pitch, size_t dst_slice_pitch, int width, int height, int depth,
                          icl_dtype dtype, const float* taps_x, const float* taps_y, const float* taps_z, int radius,
                          icl_border border, float constant, void* workspace, size_t workspace_bytes, void* stream) {
    if (width < 0 || height < 0 || depth < 0) return ICL_ERR_INVALID_VALUE;
    if (!dtype_ok(dtype)) return ICL_ERR_DTYPE;
    if (radius < 0 || radius > ICL_MAX_RADIUS_3D) return ICL_ERR_RADIUS;
    if (border != ICL_BORDER_CLAMP && border != ICL_BORDER_CONSTANT) return ICL_ERR_INVALID_VALUE;
    if (width == 0 || height == 0 || depth == 0) return ICL_OK;
    const int es = elem_size(dtype);
    icl_status s;
    if ((s = check_image(src, src_row_pitch, width, es)) != ICL_OK) return s;
    if ((s = check_image(dst, dst_row_pitch, width, es)) != ICL_OK) return s;
    const size_t sslice = (size_t)(height - 1) * src_row_pitch + (size_t)width * es;
    const size_t dslice = (size_t)(height - 1) * dst_row_pitch + (size_t)width * es;
    if (src_slice_pitch < sslice || src_slice_pitch % es || dst_slice_pitch < dslice || dst_slice_pitch % es)
        return ICL_ERR_PITCH;
    if (!taps_x || !taps_y || !taps_z) return ICL_ERR_INVALID_VALUE;
    const size_t sbytes = (size_t)(depth - 1) * src_slice_pitch + sslice;
    const size_t dbytes = (size_t)(depth - 1) * dst_slice_pitch + dslice;
    if (range_overlaps(src, sbytes, dst, dbytes)) return ICL_ERR_ALIAS;
    if (workspace && workspace_bytes &&
        (range_overlaps(workspace, workspace_bytes, src, sbytes) || range_overlaps(workspace, workspace_bytes, dst, dbytes)))
        return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    Sep3Args a{src, src_row_pitch, src_slice_pitch, dst, dst_row_pitch, dst_slice_pitch, width, height, depth,
               dtype, taps_x, taps_y, taps_z, radius, workspace, workspace_bytes, (hipStream_t)stream,
               border_of(border, constant)};
    int count;
    const Variant<Sep3Args>* tab = sep3d_variants(&count);
    const int deflt = sep3d_default(a);
    const int v = select_variant(Problem{ICL_OP_CONV3D_SEP, dtype, radius, width, height, depth}, deflt, a.st);
    const bool forced_plain = variant_forced(ICL_OP_CONV3D_SEP) && v == 0;
    if ((forced_plain || !tab[deflt].supports(a)) && !tab[0].supports(a)) return ICL_ERR_WORKSPACE;
    return dispatch(ICL_OP_CONV3D_SEP, tab, count, a, v, deflt);
}

icl_status icl_conv2d_u8(const uint8_t* src, size_t src_pitch, uint8_t* dst, size_t dst_pitch, int width,
                         int height, const int16_t* taps, int radius, int shift, icl_border border, int constant,
                         void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (radius < 0 || radius > ICL_MAX_U8_RADIUS) return ICL_ERR_RADIUS;
    if (shift < 0 || shift > ICL_MAX_U8_SHIFT) return ICL_ERR_INVALID_VALUE;
    if (border != ICL_BORDER_CLAMP && border != ICL_BORDER_CONSTANT) return ICL_ERR_INVALID_VALUE;
    if (border == ICL_BORDER_CONSTANT && (constant < 0 || constant > 255)) return ICL_ERR_INVALID_VALUE;
    if (width == 0 || height == 0) return ICL_OK;
    icl_status s;
    if ((s = check_image(src, src_pitch, width, 1)) != ICL_OK) return s;
    if ((s = check_image(dst, dst_pitch, width, 1)) != ICL_OK) return s;
    if (!taps) return ICL_ERR_INVALID_VALUE;
    if (overlaps(src, src_pitch, 1, dst, dst_pitch, 1, width, height)) return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    const int cmode = border == ICL_BORDER_CONSTANT ? 1 : 0;
    U8Args a{src, src_pitch, dst, dst_pitch, width, height, taps, radius, shift, cmode, cmode ? constant : 0,
             (hipStream_t)stream};
    int count;
    const Variant<U8Args>* tab = conv2d_u8_variants(&count);
    const int deflt = conv2d_u8_default(a);
    return dispatch(ICL_OP_CONV2D_U8, tab, count, a,
                    select_variant(ICL_OP_CONV2D_U8, ICL_U8, radius, width, height, deflt, a.st), deflt);
}

icl_status icl_harris(const float* src, size_t src_pitch, float* resp, size_t resp_pitch, int width, int height,
                      const float* window_taps, int window_radius, float k, void* workspace, size_t workspace_bytes,
                      void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (window_radius < 0 || window_radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
    if (width == 0 || height == 0) return ICL_OK;
    icl_status s;
    if ((s = check_image(src, src_pitch, width, 4)) != ICL_OK) return s;
    if ((s = check_image(resp, resp_pitch, width, 4)) != ICL_OK) return s;
    if (!window_taps) return ICL_ERR_INVALID_VALUE;
    if (overlaps(src, src_pitch, 4, resp, resp_pitch, 4, width, height)) return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    HarrisArgs a{src, src_pitch, resp, resp_pitch, width, height, window_taps, window_radius, k,
                 workspace, workspace_bytes, (hipStream_t)stream};
    int count;
    const Variant<HarrisArgs>* tab = harris_variants(&count);
    const int deflt = harris_default(a);
    const int v = select_variant(ICL_OP_HARRIS, ICL_F32, window_radius, width, height, deflt, a.st);
    const bool forced_split = variant_forced(ICL_OP_HARRIS) && v == 0;
    if ((forced_split || !tab[deflt].supports(a)) && !tab[0].supports(a)) return ICL_ERR_WORKSPACE;
    return dispatch(ICL_OP_HARRIS, tab, count, a, v, deflt);
}

icl_status icl_nms(const float* resp, size_t resp_pitch, uint8_t* mask, size_t mask_pitch, int width, int height,
                   int radius, float threshold, void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (radius < 1 || radius > ICL_MAX_NMS_RADIUS) return ICL_ERR_RADIUS;
    if (width == 0 || height == 0) return ICL_OK;
    icl_status s;
    if ((s = check_image(resp, resp_pitch, width, 4)) != ICL_OK) return s;
    if ((s = check_image(mask, mask_pitch, width, 1)) != ICL_OK) return s;
    if (overlaps(resp, resp_pitch, 4, mask, mask_pitch, 1, width, height)) return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    NmsArgs a{resp, resp_pitch, mask, mask_pitch, width, height, radius, threshold, (hipStream_t)stream};
    int count;
    const Variant<NmsArgs>* tab = nms_variants(&count);
    const int deflt = nms_default(a);
    return dispatch(ICL_OP_NMS, tab, count, a, select_variant(ICL_OP_NMS, ICL_F32, radius, width, height, deflt, a.st), deflt);
}

// ------------------------------------------------------------------ filter bank
icl_status icl_corners(const float* src, size_t src_pitch, uint8_t* mask, size_t mask_pitch, int width, int height,
                       const float* window_taps, int window_radius, float k, int nms_radius, float threshold,
                       float* resp, size_t resp_pitch, void* workspace, size_t workspace_bytes, void* stream) {
    if (width < 0 || height < 0) return ICL_ERR_INVALID_VALUE;
    if (window_radius < 0 || window_radius > ICL_MAX_WINDOW_RADIUS) return ICL_ERR_RADIUS;
    if (nms_radius < 1 || nms_radius > ICL_MAX_NMS_RADIUS) return ICL_ERR_RADIUS;
    if (width == 0 || height == 0) return ICL_OK;
    icl_status s;
    if ((s = check_image(src, src_pitch, width, 4)) != ICL_OK) return s;
    if ((s = check_image(mask, mask_pitch, width, 1)) != ICL_OK) return s;
    if (resp && (s = check_image(resp, resp_pitch, width, 4)) != ICL_OK) return s;
    if (!window_taps) return ICL_ERR_INVALID_VALUE;
    if (overlaps(src, src_pitch, 4, mask, mask_pitch, 1, width, height)) return ICL_ERR_ALIAS;
    if (resp && (overlaps(src, src_pitch, 4, resp, resp_pitch, 4, width, height) ||
                 overlaps(mask, mask_pitch, 1, resp, resp_pitch, 4, width, height)))
        return ICL_ERR_ALIAS;
    if (workspace && workspace_bytes) {
        const size_t sb = (size_t)(height - 1) * src_pitch + (size_t)width * 4;
        const size_t mb = (size_t)(height - 1) * mask_pitch + (size_t)width;
        const size_t rb = (size_t)(height - 1) * resp_pitch + (size_t)width * 4;
        if (range_overlaps(workspace, workspace_bytes, src, sb) || range_overlaps(workspace, workspace_bytes, mask, mb) ||
            (resp && range_overlaps(workspace, workspace_bytes, resp, rb)))
            return ICL_ERR_ALIAS;
    }
    if ((s = device_ready()) != ICL_OK) return s;
    CornersArgs a{src, src_pitch, mask, mask_pitch, width, height, window_taps, window_radius, k, nms_radius,
                  threshold, resp, resp ? resp_pitch : 0, workspace, workspace_bytes, (hipStream_t)stream};
    int count;
    const Variant<CornersArgs>* tab = corners_variants(&count);
    const int deflt = corners_default(a);
    const int v = select_variant(ICL_OP_CORNERS, ICL_F32, window_radius, width, height, deflt, a.st);
    // the two-kernel variant needs somewhere to put the response
    const bool forced_two = variant_forced(ICL_OP_CORNERS) && v == 0;
    if ((forced_two || !tab[deflt].supports(a)) && !tab[0].supports(a)) return ICL_ERR_WORKSPACE;
    return dispatch(ICL_OP_CORNERS, tab, count, a, v, deflt);
}

static icl_status check_bank(int n, int f, int h, int wd, int radius) {
    if (n < 0 || f < 1 || h < 0 || wd < 0) return ICL_ERR_INVALID_VALUE;
    if (f > 64) return ICL_ERR_UNSUPPORTED;
    if (radius < 1 || radius > 4) return ICL_ERR_RADIUS;
    return ICL_OK;
}

icl_status icl_bank_fwd(const float* x, const float* w, float* y, int n, int f, int h, int wd, int radius,
                        void* stream) {
    icl_status s;
    if ((s = check_bank(n, f, h, wd, radius)) != ICL_OK) return s;
    if (n == 0 || h == 0 || wd == 0) return ICL_OK;
    if (!x || !w || !y) return ICL_ERR_INVALID_VALUE;
    const size_t hw = (size_t)h * wd;
    if (range_overlaps(x, (size_t)n * hw * 4, y, (size_t)n * f * hw * 4) ||
        range_overlaps(w, (size_t)f * (2 * radius + 1) * (2 * radius + 1) * 4, y, (size_t)n * f * hw * 4))
        return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    BankArgs a{x, w, y, n, f, h, wd, radius, nullptr, 0, (hipStream_t)stream};
    int count;
    const Variant<BankArgs>* tab = bank_fwd_variants(&count);
    const int deflt = bank_fwd_default(a);
    return dispatch(ICL_OP_BANK_FWD, tab, count, a, select_variant(Problem{ICL_OP_BANK_FWD, ICL_F32, radius, wd, h, 1, n, f}, deflt, a.st),
                    deflt);
}

icl_status icl_bank_bwd_input(const float* gy, const float* w, float* gx, int n, int f, int h, int wd, int radius,
                              const float* scale, void* stream) {
    icl_status s;
    if ((s = check_bank(n, f, h, wd, radius)) != ICL_OK) return s;
    if (n == 0 || h == 0 || wd == 0) return ICL_OK;
    if (!gy || !w || !gx) return ICL_ERR_INVALID_VALUE;
    const size_t hw = (size_t)h * wd;
    if (range_overlaps(gy, (size_t)n * f * hw * 4, gx, (size_t)n * hw * 4) ||
        range_overlaps(w, (size_t)f * (2 * radius + 1) * (2 * radius + 1) * 4, gx, (size_t)n * hw * 4))
        return ICL_ERR_ALIAS;
    if (scale && range_overlaps(scale, 4, gx, (size_t)n * hw * 4)) return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    BankArgs a{gy, w, gx, n, f, h, wd, radius, nullptr, 0, (hipStream_t)stream, scale};
    int count;
    const Variant<BankArgs>* tab = bank_bwd_input_variants(&count);
    const int deflt = bank_bwd_input_default(a);
    return dispatch(ICL_OP_BANK_BWD_INPUT, tab, count, a,
                    select_variant(Problem{ICL_OP_BANK_BWD_INPUT, ICL_F32, radius, wd, h, 1, n, f}, deflt, a.st), deflt);
}

icl_status icl_bank_bwd_filter(const float* gy, const float* x, float* gw, int n, int f, int h, int wd, int radius,
                               const float* scale, void* workspace, size_t workspace_bytes, void* stream) {
    icl_status s;
    if ((s = check_bank(n, f, h, wd, radius)) != ICL_OK) return s;
    if (!gw) return ICL_ERR_INVALID_VALUE;
    const size_t nk = (size_t)(2 * radius + 1) * (2 * radius + 1);
    if (n == 0 || h == 0 || wd == 0) {
        if ((s = device_ready()) != ICL_OK) return s;
        return hip_status(zero_fill(gw, (size_t)f * nk, (hipStream_t)stream));
    }
    if (!gy || !x) return ICL_ERR_INVALID_VALUE;
    const size_t need = bank_bwd_filter_workspace(n, f, h, wd, radius);
    if (!workspace || workspace_bytes < need) return ICL_ERR_WORKSPACE;
    const size_t hw = (size_t)h * wd;
    if (range_overlaps(gw, (size_t)f * nk * 4, gy, (size_t)n * f * hw * 4) ||
        range_overlaps(gw, (size_t)f * nk * 4, x, (size_t)n * hw * 4) ||
        range_overlaps(workspace, need, gy, (size_t)n * f * hw * 4) ||
        range_overlaps(workspace, need, x, (size_t)n * hw * 4) || range_overlaps(workspace, need, gw, (size_t)f * nk * 4))
        return ICL_ERR_ALIAS;
    if (scale && (range_overlaps(scale, 4, gw, (size_t)f * nk * 4) || range_overlaps(scale, 4, workspace, need)))
        return ICL_ERR_ALIAS;
    if ((s = device_ready()) != ICL_OK) return s;
    BankArgs a{gy, x, gw, n, f, h, wd, radius, workspace, workspace_bytes, (hipStream_t)stream, scale};
    int count;
    const Variant<BankArgs>* tab = bank_bwd_filter_variants(&count);
    const int deflt = bank_bwd_filter_default(a);
    return dispatch(ICL_OP_BANK_BWD_FILTER, tab, count, a,
                    select_variant(Problem{ICL_OP_BANK_BWD_FILTER, ICL_F32, radius, wd, h, 1, n, f}, deflt, a.st), deflt);
}

icl_status icl_sse_loss(const float* y, const float* t, float* gy, long long count, float* loss, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (count < 0) return ICL_ERR_INVALID_VALUE;
    if (!loss) return ICL_ERR_INVALID_VALUE;
    if (count > 0 && (!y || !t)) return ICL_ERR_INVALID_VALUE;
    if (!workspace || workspace_bytes < sse_workspace(count)) return ICL_ERR_WORKSPACE;
    const size_t nb = (size_t)count * 4;
    if (gy && (range_overlaps(gy, nb, y, nb) || range_overlaps(gy, nb, t, nb))) return ICL_ERR_ALIAS;
    icl_status s;
    if ((s = device_ready()) != ICL_OK) return s;
    return hip_status(sse_launch(y, t, gy, count, loss, workspace, workspace_bytes, (hipStream_t)stream));
}

}  // extern "C"

namespace icl {

// The fused forward + loss entry point.
// may_tune: whether a tune-cache miss may start a search (ICL_TUNE=search); a search
// allocates, so the allocation-free entry point passes false.
icl_status bank_fwd_sse_entry(const float* x, const float* w, const float* t, float* y, float* gy, float* loss, int n,
                              int f, int h, int wd, int radius, void* workspace, size_t workspace_bytes,
                              void* stream, bool may_tune) {
    icl_status s;
    if ((s = check_bank(n, f, h, wd, radius)) != ICL_OK) return s;
    if (!loss) return ICL_ERR_INVALID_VALUE;
    if (!workspace || workspace_bytes < bank_fwd_sse_workspace()) return ICL_ERR_WORKSPACE;
    const size_t hw = (size_t)h * wd, nx = (size_t)n * hw * 4, ny = (size_t)n * f * hw * 4;
    const size_t nw = (size_t)f * (2 * radius + 1) * (2 * radius + 1) * 4;
    if (ny > 0 && (!x || !w || !t)) return ICL_ERR_INVALID_VALUE;
    // outputs against every input and against each other (the loss scalar and the workspace too)
    const void* outs[4] = {y, gy, loss, workspace};
    const size_t onb[4] = {ny, ny, 4, workspace_bytes};
    const void* ins[3] = {x, w, t};
    const size_t inb[3] = {nx, nw, ny};
    for (int i = 0; i < 4; ++i) {
        if (!outs[i] || !onb[i]) continue;
        for (int j = 0; j < 3; ++j)
            if (ins[j] && inb[j] && range_overlaps(outs[i], onb[i], ins[j], inb[j])) return ICL_ERR_ALIAS;
        for (int j = i + 1; j < 4; ++j)
            if (outs[j] && onb[j] && range_overlaps(outs[i], onb[i], outs[j], onb[j])) return ICL_ERR_ALIAS;
    }
    if ((s = device_ready()) != ICL_OK) return s;
    BankSseArgs a{x, w, t, y, gy, loss, n, f, h, wd, radius, workspace, workspace_bytes, (hipStream_t)stream};
    if (ny == 0) {   // empty batch: L = 0
        return hip_status(zero_fill(loss, 1, a.st));
    }
    int count;
    const Variant<BankSseArgs>* tab = bank_fwd_sse_variants(&count);
    const int deflt = bank_fwd_sse_default(a);
    const int v = select_variant(Problem{ICL_OP_BANK_FWD_SSE, ICL_F32, radius, wd, h, 1, n, f}, deflt,
                                 may_tune ? a.st : nullptr);
    return dispatch(ICL_OP_BANK_FWD_SSE, tab, count, a, v, deflt);
}

// ------------------------------------------------------------------ fixed device scratch
// The loss partials of icl_bank_fwd_sse_noalloc live in this array, one copy per device,
// held until the process ends.  Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address): it looks up each device's address
// once, with that device current, and passes that.
constexpr size_t kScratchBytes = FWD_SSE_PARTS * sizeof(double);
static __device__ __align__(256) double scratch[FWD_SSE_PARTS];
static_assert(sizeof(scratch) == kScratchBytes, "scratch holds the fused loss partials");

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (null and the HIP error recorded when
// the lookup fails).
static void* scratch_on_current_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e);
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            set_hip_error(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace icl

extern "C" {

icl_status icl_bank_fwd_sse(const float* x, const float* w, const float* t, float* y, float* gy, float* loss, int n,
                            int f, int h, int wd, int radius, void* workspace, size_t workspace_bytes, void* stream) {
    return bank_fwd_sse_entry(x, w, t, y, gy, loss, n, f, h, wd, radius, workspace, workspace_bytes, stream, true);
}

icl_status icl_bank_fwd_sse_noalloc(const float* x, const float* w, const float* t, float* y, float* gy, float* loss,
                                    int n, int f, int h, int wd, int radius, void* stream) {
    icl_status s = device_ready();
    if (s != ICL_OK) return s;
    if (bank_fwd_sse_workspace() > kScratchBytes) return ICL_ERR_WORKSPACE;
    void* ws = scratch_on_current_device();
    if (!ws) return ICL_ERR_HIP;
    return bank_fwd_sse_entry(x, w, t, y, gy, loss, n, f, h, wd, radius, ws, kScratchBytes, stream, false);
}

// ------------------------------------------------------------------ variants
int icl_variant_count(icl_op op) {
    int c = 0;
    switch (op) {
        case ICL_OP_CONV_SEP: sep_variants(&c); break;
        case ICL_OP_CONV2D: conv2d_variants(&c); break;
        case ICL_OP_CONV2D_U8: conv2d_u8_variants(&c); break;
        case ICL_OP_CORNERS: corners_variants(&c); break;
        case ICL_OP_CONV3D_SEP: sep3d_variants(&c); break;
        case ICL_OP_HARRIS: harris_variants(&c); break;
        case ICL_OP_NMS: nms_variants(&c); break;
        case ICL_OP_BANK_FWD: bank_fwd_variants(&c); break;
        case ICL_OP_BANK_BWD_INPUT: bank_bwd_input_variants(&c); break;
        case ICL_OP_BANK_BWD_FILTER: bank_bwd_filter_variants(&c); break;
        case ICL_OP_BANK_FWD_SSE: bank_fwd_sse_variants(&c); break;
        case ICL_OP_CONV_SEP_BATCHED: c = 11; break;
        case ICL_OP_SSE_LOSS: c = 1; break;
        default: c = 0;
    }
    return c;
}

const char* icl_variant_name(icl_op op, int index) {
    if (index < 0 || index >= icl_variant_count(op)) return nullptr;
    int c = 0;
    switch (op) {
        case ICL_OP_CONV_SEP: return sep_variants(&c)[index].name;
        case ICL_OP_CONV2D: return conv2d_variants(&c)[index].name;
        case ICL_OP_CONV2D_U8: return conv2d_u8_variants(&c)[index].name;
        case ICL_OP_CORNERS: return corners_variants(&c)[index].name;
        case ICL_OP_CONV3D_SEP: return sep3d_variants(&c)[index].name;
        case ICL_OP_HARRIS: return harris_variants(&c)[index].name;
        case ICL_OP_NMS: return nms_variants(&c)[index].name;
        case ICL_OP_BANK_FWD: return bank_fwd_variants(&c)[index].name;
        case ICL_OP_BANK_BWD_INPUT: return bank_bwd_input_variants(&c)[index].name;
        case ICL_OP_BANK_BWD_FILTER: return bank_bwd_filter_variants(&c)[index].name;
        case ICL_OP_BANK_FWD_SSE: return bank_fwd_sse_variants(&c)[index].name;
        case ICL_OP_CONV_SEP_BATCHED: {
            static const char* names[] = {"persistent_fused_t64", "persistent_strip_t32",
                                          "persistent_fused_t64_rsort", "persistent_fused_t32_rsort",
                                          "colwalk_s256", "colwalk_s512", "colwalk_s2048", "colwalk_s128",
                                          "colwalk_s64", "colwalk128_s128", "colwalk128_s256"};
            return names[index];
        }
        case ICL_OP_SSE_LOSS: return "two_stage";
        default: return nullptr;
    }
}

icl_status icl_set_math(icl_math mode) {
    if (mode != ICL_MATH_F32 && mode != ICL_MATH_F16_SPLIT) return ICL_ERR_INVALID_VALUE;
    g_math = (int)mode;
    return ICL_OK;
}

icl_math icl_get_math(void) { return (icl_math)g_math.load(); }

const char* icl_variant_arith(icl_op op, int index) { return arith_of(op, icl_variant_name(op, index)); }

icl_status icl_force_variant(icl_op op, int index) {
    if (op < 0 || op >= ICL_OP_COUNT) return ICL_ERR_INVALID_VALUE;
    if (index < -1 || index >= icl_variant_count(op)) return ICL_ERR_INVALID_VALUE;
    ensure_force_env();
    g_forced[op] = index;
    return ICL_OK;
}

icl_status icl_selected_variant(icl_op op, icl_dtype dtype, int radius, int width, int height, int* index) {
    const icl_problem q{op, dtype, radius, width, height, 1, 1, 1};
    return icl_selected_variant_problem(&q, index);
}

icl_status icl_selected_variant_problem(const icl_problem* q, int* index) {
    if (!index || !q || q->op < 0 || q->op >= ICL_OP_COUNT) return ICL_ERR_INVALID_VALUE;
    const icl_op op = q->op;
    const icl_dtype dtype = q->dtype;
    const int radius = q->radius, width = q->width, height = q->height;
    int deflt = 0;
    switch (op) {
        case ICL_OP_CONV_SEP: {
            SepArgs a{};
            a.r = radius; a.W = width; a.H = height; a.dt = dtype;
            deflt = sep_default(a);
            break;
        }
        case ICL_OP_CONV2D: {
            Conv2dArgs a{};
            a.r = radius;
            deflt = conv2d_default(a);
            break;
        }
        case ICL_OP_HARRIS: {
            HarrisArgs a{};
            a.rg = radius;
            deflt = harris_default(a);
            break;
        }
        case ICL_OP_NMS: {
            NmsArgs a{};
            a.r = radius;
            deflt = nms_default(a);
            break;
        }
        case ICL_OP_CONV_SEP_BATCHED: deflt = batched_default(); break;
        case ICL_OP_CONV2D_U8: {
            U8Args a{};
            a.r = radius;
            deflt = conv2d_u8_default(a);
            break;
        }
        case ICL_OP_CONV3D_SEP: {
            Sep3Args a{};
            a.r = radius;
            deflt = sep3d_default(a);
            break;
        }
        case ICL_OP_CORNERS: {
            CornersArgs a{};
            a.rg = radius;
            a.nr = 1;
            deflt = corners_default(a);
            break;
        }
        case ICL_OP_BANK_FWD: case ICL_OP_BANK_BWD_INPUT: case ICL_OP_BANK_BWD_FILTER: {
            BankArgs a{};
            a.n = q->n; a.f = q->f; a.h = height; a.w = width; a.r = radius;
            deflt = op == ICL_OP_BANK_FWD ? bank_fwd_default(a)
                    : op == ICL_OP_BANK_BWD_INPUT ? bank_bwd_input_default(a) : bank_bwd_filter_default(a);
            break;
        }
        case ICL_OP_BANK_FWD_SSE: {
            BankSseArgs a{};
            a.n = q->n; a.f = q->f; a.h = height; a.wd = width; a.r = radius;
            deflt = bank_fwd_sse_default(a);
            break;
        }
        default: break;
    }
    *index = select_variant(problem_of(*q), deflt);
    return ICL_OK;
}

}  // extern "C"
