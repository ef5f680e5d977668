// Device-side helpers shared by the gfx950 stencil kernels: storage decode /
// encode, clamped indexing and work-group ordering.
#pragma once
#include <type_traits>
#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icl {

// Calls f(std::integral_constant<int, 0>{}) ... f(integral_constant<int, N-1>{}): a loop whose
// index is a compile-time constant in the body (static register-ring slots).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// What a read outside the image returns: the closest pixel inside (clamp, the default) or
// a constant value (Section 5, Fig. 3).
struct Border {
    int constant = 0;   // 0: clamp, 1: constant
    float value = 0.f;
};

// Neighbour-lane moves within a wave as DPP wave shifts (a VALU operand modifier, no LDS
// round trip): lane i receives v of lane i-1 (from_left) or of lane i+1 (from_right); the
// end lane with no such neighbour receives 0.
__device__ __forceinline__ float lane_from_left(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}

// The same shifts with the end lane's value supplied: lane 0 (from_left) or lane 63
// (from_right) receives `edge`.  One DPP move whose old value is `edge` (bound_ctrl off: a
// lane without a source keeps the old value), with every lane active.  (A select on the lane
// index around a plain shift is not equivalent: the compiler may turn it into a branch that
// masks the end lane off, and a DPP read from a masked-off lane yields 0 for its neighbour.)
__device__ __forceinline__ float lane_from_left_or(float v, float edge) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_from_right_or(float v, float edge) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// Native 4 x float32 vector: loads and stores of it lower to single dwordx4 /
// ds_read_b128 instructions (HIP's float4 struct is copied member by member).
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mk4(float a, float b, float c, float d) { return v4f{a, b, c, d}; }
__device__ __forceinline__ v4f lds4(const float* p) { return *reinterpret_cast<const v4f*>(p); }
__device__ __forceinline__ void lds4(float* p, v4f v) { *reinterpret_cast<v4f*>(p) = v; }

// ------------------------------------------------------------------ storage types
// Pixel storage tags.  Arithmetic is always float32; these convert on load/store.
struct F32 { using storage = float; static constexpr int size = 4; };
struct F16 { using storage = _Float16; static constexpr int size = 2; };
struct BF16 { using storage = uint16_t; static constexpr int size = 2; };

__device__ __forceinline__ float decode(float v) { return v; }
__device__ __forceinline__ float decode(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float decode_bf16(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// bfloat16 round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t encode_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

template <class T> __device__ __forceinline__ float load_px(const void* base, size_t off_bytes);
template <> __device__ __forceinline__ float load_px<F32>(const void* base, size_t off) {
    return *reinterpret_cast<const float*>(static_cast<const char*>(base) + off);
}
template <> __device__ __forceinline__ float load_px<F16>(const void* base, size_t off) {
    return decode(*reinterpret_cast<const _Float16*>(static_cast<const char*>(base) + off));
}
template <> __device__ __forceinline__ float load_px<BF16>(const void* base, size_t off) {
    return decode_bf16(*reinterpret_cast<const uint16_t*>(static_cast<const char*>(base) + off));
}

template <class T> __device__ __forceinline__ void store_px(void* base, size_t off, float v);
template <> __device__ __forceinline__ void store_px<F32>(void* base, size_t off, float v) {
    *reinterpret_cast<float*>(static_cast<char*>(base) + off) = v;
}
// float32 -> float16, round to nearest even, from a float32 value that is final: the
// empty asm keeps the compiler from merging the conversion with the FMA that produced v
// (a mixed-precision FMA would round once, straight to float16, and differ from the
// float32-then-float16 rounding of every other kernel in rare cases).
__device__ __forceinline__ _Float16 encode_f16(float v) {
    asm volatile("" : "+v"(v));
    return static_cast<_Float16>(v);
}

template <> __device__ __forceinline__ void store_px<F16>(void* base, size_t off, float v) {
    *reinterpret_cast<_Float16*>(static_cast<char*>(base) + off) = encode_f16(v);
}
template <> __device__ __forceinline__ void store_px<BF16>(void* base, size_t off, float v) {
    *reinterpret_cast<uint16_t*>(static_cast<char*>(base) + off) = encode_bf16(v);
}

// Four consecutive pixels starting at a byte offset that is 4*size aligned.
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

template <class T> __device__ __forceinline__ v4f load4(const void* base, size_t off);
template <> __device__ __forceinline__ v4f load4<F32>(const void* base, size_t off) {
    return *reinterpret_cast<const v4f*>(static_cast<const char*>(base) + off);
}
template <> __device__ __forceinline__ v4f load4<F16>(const void* base, size_t off) {
    const v4h h = *reinterpret_cast<const v4h*>(static_cast<const char*>(base) + off);
    return v4f{decode(h.x), decode(h.y), decode(h.z), decode(h.w)};
}
template <> __device__ __forceinline__ v4f load4<BF16>(const void* base, size_t off) {
    const v2u u = *reinterpret_cast<const v2u*>(static_cast<const char*>(base) + off);
    return v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
               __uint_as_float(u.y & 0xffff0000u)};
}

template <class T> __device__ __forceinline__ void store4(void* base, size_t off, v4f v);
template <> __device__ __forceinline__ void store4<F32>(void* base, size_t off, v4f v) {
    *reinterpret_cast<v4f*>(static_cast<char*>(base) + off) = v;
}
template <> __device__ __forceinline__ void store4<F16>(void* base, size_t off, v4f v) {
    const v4h h = {encode_f16(v.x), encode_f16(v.y), encode_f16(v.z), encode_f16(v.w)};
    *reinterpret_cast<v4h*>(static_cast<char*>(base) + off) = h;
}
template <> __device__ __forceinline__ void store4<BF16>(void* base, size_t off, v4f v) {
    v2u u;
    u.x = static_cast<uint32_t>(encode_bf16(v.x)) | (static_cast<uint32_t>(encode_bf16(v.y)) << 16);
    u.y = static_cast<uint32_t>(encode_bf16(v.z)) | (static_cast<uint32_t>(encode_bf16(v.w)) << 16);
    *reinterpret_cast<v2u*>(static_cast<char*>(base) + off) = u;
}

// ------------------------------------------------------------------ buffer-descriptor access
// A raw buffer descriptor (base, size in bytes) lets a lane address the buffer with a 32-bit
// byte offset (one VALU add instead of 64-bit address arithmetic), and the hardware's range
// check returns 0 for a load at or past the size (and drops such a store) without touching
// memory.  Dword 3 is the gfx9-family format word for untyped raw access.
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Four pixels of storage type T at a byte offset, as stored (float32: four floats; half
// types: four 16-bit values packed in two dwords), and their float32 values.
template <class T> struct Raw4 { using type = v2u; };
template <> struct Raw4<F32> { using type = v4f; };
template <class T> __device__ __forceinline__ typename Raw4<T>::type bload4_raw(Rsrc rs, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
}
template <> __device__ __forceinline__ v4f bload4_raw<F32>(Rsrc rs, unsigned off) {
    return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
}
// one pixel's stored bits, zero-extended
template <class T> __device__ __forceinline__ unsigned bload1_raw(Rsrc rs, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
}
template <> __device__ __forceinline__ unsigned bload1_raw<F32>(Rsrc rs, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
}
// four single pixels' bits (each zero-extended) packed as bload4_raw would return them
template <class T> __device__ __forceinline__ typename Raw4<T>::type pack4_raw(unsigned a, unsigned b, unsigned c,
                                                                              unsigned d) {
    return v2u{a | (b << 16), c | (d << 16)};
}
template <> __device__ __forceinline__ v4f pack4_raw<F32>(unsigned a, unsigned b, unsigned c, unsigned d) {
    return v4f{__uint_as_float(a), __uint_as_float(b), __uint_as_float(c), __uint_as_float(d)};
}
template <class T> __device__ __forceinline__ v4f decode4(typename Raw4<T>::type r);
template <> __device__ __forceinline__ v4f decode4<F32>(v4f r) { return r; }
template <> __device__ __forceinline__ v4f decode4<F16>(v2u r) {
    const v4h h = __builtin_bit_cast(v4h, r);
    return v4f{decode(h.x), decode(h.y), decode(h.z), decode(h.w)};
}
template <> __device__ __forceinline__ v4f decode4<BF16>(v2u r) {
    return v4f{__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u), __uint_as_float(r.y << 16),
               __uint_as_float(r.y & 0xffff0000u)};
}

// ------------------------------------------------------------------ indexing
// Closest in-range index along one axis (clamped boundary condition).
__device__ __forceinline__ int clampi(int i, int n) { return min(max(i, 0), n - 1); }

// Work-group order that keeps consecutive logical tiles on one XCD.  gfx950
// dispatches work-groups round-robin over its 8 XCDs (each with a private L2), so
// logical tile t is taken by the block whose hardware id places it on XCD t/(n/8).
// Neighbouring tiles share halo rows; keeping them on one XCD serves the halo
// from that XCD's L2.  Falls back to identity when n is not a multiple of 8.
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned n) {
    if (n % 8u) return bid;
    return (bid % 8u) * (n / 8u) + bid / 8u;
}

// Grid padded to a multiple of 8 (xcd_remap is a permutation of such a grid).
inline unsigned grid_pad8(long long n) { return (unsigned)((n + 7) / 8 * 8); }

}  // namespace icl
