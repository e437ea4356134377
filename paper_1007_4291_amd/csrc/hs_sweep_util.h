// Definitions shared by the sweep kernels (a3 / a4): compile-time loops, stored-column chunks,
// conversions, lane sums and the prefetch depth.
#pragma once

#include <utility>

#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>): a loop unrolled at compile time
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

enum SweepMode : int { MODE_FWD = 0, MODE_BWD = 1, MODE_MID = 2, MODE_SUB = 3 };

// 16-byte chunk of a stored factor column (native vector type, kept in registers by the compiler)
typedef unsigned int chunk16 __attribute__((ext_vector_type(4)));

template <class TF, int BS> struct ColChunks {
    static constexpr int STRIDE = col_stride<TF>(BS);
    static constexpr int N16 = STRIDE * (int)sizeof(C2<TF>) / 16;   // 16-byte chunks per column
    static constexpr int NCH = (N16 + 63) / 64;                      // chunks per lane
};

__device__ __forceinline__ double2 ld2(const HS_GLOBAL double2* p) { return gld(p); }
__device__ __forceinline__ double2 ld2(const HS_GLOBAL float2* p) { const float2 v = gld(p); return make_double2(v.x, v.y); }
template <class TO, class T> __device__ __forceinline__ TO cvt_out(C2<T> v);
template <> __device__ __forceinline__ double2 cvt_out<double2, double>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 cvt_out<double2, float>(float2 v) { return make_double2(v.x, v.y); }
template <> __device__ __forceinline__ float2 cvt_out<float2, float>(float2 v) { return v; }
template <> __device__ __forceinline__ float2 cvt_out<float2, double>(double2 v) { return make_float2((float)v.x, (float)v.y); }

struct SubArg {
    const void* fac;
    const double2* g;
    double2* x;
    const double2* ris2;    // 1/s2 of local row r at ris2[rstep * r]
    int nrhs, rstep, cdir, jl;
};

// Sum of v over lanes l and l ^ OFF (OFF = 16 or 32), in every lane, with the gfx950 row / half-wave
// swap instructions (no LDS round trip).
template <int OFF> __device__ __forceinline__ float xor_sum(float v) {
    const unsigned b = __float_as_uint(v);
    const auto s = OFF == 16 ? __builtin_amdgcn_permlane16_swap(b, b, false, false)
                             : __builtin_amdgcn_permlane32_swap(b, b, false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
template <int OFF> __device__ __forceinline__ double xor_sum(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    const auto sl = OFF == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                              : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto sh = OFF == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                              : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double a = __longlong_as_double((long long)(((uint64_t)sh[0] << 32) | sl[0]));
    const double c = __longlong_as_double((long long)(((uint64_t)sh[1] << 32) | sl[1]));
    return a + c;
}

// Raw buffer access: a wave-uniform resource (base, size in bytes) plus a per-lane byte offset in a
// VGPR and a wave-uniform byte offset in an SGPR, so per-step address arithmetic stays scalar.
typedef unsigned int hs_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const HS_GLOBAL void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)base, (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ chunk16 buf_ld16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_ld(float2& v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const hs_u2 b = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    v = make_float2(__uint_as_float(b.x), __uint_as_float(b.y));
}
__device__ __forceinline__ void buf_ld(double2& v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const chunk16 b = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    v = make_double2(__hiloint2double((int)b.y, (int)b.x), __hiloint2double((int)b.w, (int)b.z));
}
__device__ __forceinline__ void buf_st(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    hs_u2 b;
    b.x = __float_as_uint(v.x); b.y = __float_as_uint(v.y);
    __builtin_amdgcn_raw_buffer_store_b64(b, r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const uint64_t a = (uint64_t)__double_as_longlong(v.x), c = (uint64_t)__double_as_longlong(v.y);
    chunk16 b;
    b.x = (unsigned)a; b.y = (unsigned)(a >> 32); b.z = (unsigned)c; b.w = (unsigned)(c >> 32);
    __builtin_amdgcn_raw_buffer_store_b128(b, r, (int)voff, (int)soff, 0);
}

// acc += l * z_k for complex values, where z_k is lane k of this lane's 16-lane row (DPP row
// broadcast as the first operand of each fused multiply-add: no LDS round trip for the vector).  The
// leading s_nop covers the two wait states between a VALU write of z and its read through DPP.  Not
// volatile: the compiler may schedule the loads of l ahead of it.
template <int K>
__device__ __forceinline__ void cfma_rowbcast(float& ax, float& ay, float lx, float ly, float zx, float zy) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %4, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %5, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%5, %3 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %3 row_newbcast:%6 row_mask:0xf bank_mask:0xf"
        : "+v"(ax), "+v"(ay)
        : "v"(lx), "v"(ly), "v"(zx), "v"(zy), "i"(K));
}
// The same product starting a sum: acc = l * z_k (no zeroed accumulators to initialise).
template <int K>
__device__ __forceinline__ void cmul_rowbcast(float& ax, float& ay, float lx, float ly, float zx, float zy) {
    asm("s_nop 1\n\t"
        "v_mul_f32_dpp %0, %4, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %5, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, -%5, %3 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %3 row_newbcast:%6 row_mask:0xf bank_mask:0xf"
        : "=&v"(ax), "=&v"(ay)
        : "v"(lx), "v"(ly), "v"(zx), "v"(zy), "i"(K));
}

// prefetch distance in ticks: as deep as the register budget of one wave allows
template <class T, int BS> struct Ring { static constexpr int D = (sizeof(T) == 8 || BS > 17) ? 2 : 4; };

}  // namespace hs
