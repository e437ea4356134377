// Shared device-side definitions of the helmsweep library (gfx950).
//
// Complex numbers are HIP vector pairs (x = re, y = im): double2 for complex128, float2 for
// complex64.  Problem, subproblem and chain descriptors live in device memory so that one launch
// can serve a whole batch of problems of different sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

// ---------------------------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------------------------
template <class T> struct c2;
template <> struct c2<double> { using t = double2; };
template <> struct c2<float> { using t = float2; };
template <class T> using C2 = typename c2<T>::t;

template <class T> __host__ __device__ __forceinline__ C2<T> mk(T re, T im) { C2<T> z; z.x = re; z.y = im; return z; }
template <class T> __host__ __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <class T> __host__ __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <class T> __host__ __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a*b
template <class T> __host__ __device__ __forceinline__ C2<T> cfma(C2<T> a, C2<T> b, C2<T> acc) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc - a*b
template <class T> __host__ __device__ __forceinline__ C2<T> cfms(C2<T> a, C2<T> b, C2<T> acc) {
    acc.x = fma(-a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// conj(a) * b
template <class T> __host__ __device__ __forceinline__ C2<T> cconjmul(C2<T> a, C2<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <class T> __host__ __device__ __forceinline__ T cabs2(C2<T> a) { return a.x * a.x + a.y * a.y; }
template <class T> __host__ __device__ __forceinline__ C2<T> cinv(C2<T> a) {
    // 1/a with scaling against overflow / underflow of |a|^2
    T s = fmax(fabs(a.x), fabs(a.y));
    T ar = a.x / s, ai = a.y / s;
    T d = s * (ar * ar + ai * ai);
    return mk<T>(ar / d, -ai / d);
}
template <class T> __host__ __device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// c ? a : b component by component (a select of the whole vector struct can be lowered through
// scratch memory)
template <class T> __host__ __device__ __forceinline__ C2<T> csel(bool c, C2<T> a, C2<T> b) {
    return mk<T>(c ? a.x : b.x, c ? a.y : b.y);
}
template <class To, class Ti> __host__ __device__ __forceinline__ C2<To> ccast(C2<Ti> a) {
    return mk<To>((To)a.x, (To)a.y);
}

// Pointers read from descriptor tables are generic; accessing device memory through them as
// global-address-space pointers gives global_load/store (counted by vmcnt only) instead of flat
// operations, whose completion also gates every LDS wait.
#define HS_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ HS_GLOBAL T* gptr(T* p) { return (HS_GLOBAL T*)p; }
template <class T> __device__ __forceinline__ const HS_GLOBAL T* gptr(const T* p) { return (const HS_GLOBAL T*)p; }
// complex loads / stores through global pointers (HIP's vector types cannot be copied across
// address spaces, so the access goes through native vector types)
typedef double hs_d2v __attribute__((ext_vector_type(2)));
typedef float hs_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gld(const HS_GLOBAL double2* p) {
    const hs_d2v v = *(const HS_GLOBAL hs_d2v*)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gld(const HS_GLOBAL float2* p) {
    const hs_f2v v = *(const HS_GLOBAL hs_f2v*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(HS_GLOBAL double2* p, double2 v) {
    hs_d2v w;
    w.x = v.x; w.y = v.y;
    *(HS_GLOBAL hs_d2v*)p = w;
}
__device__ __forceinline__ void gst(HS_GLOBAL float2* p, float2 v) {
    hs_f2v w;
    w.x = v.x; w.y = v.y;
    *(HS_GLOBAL hs_f2v*)p = w;
}

// Ordering of LDS accesses inside a workgroup of exactly one wave.  LDS operations of one wave are
// performed in issue order, so only the compiler has to be kept from moving memory accesses across
// this point; unlike __syncthreads() it does not wait for outstanding global loads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------------------------
enum SubKind : int32_t { SUB_PHYS = 0, SUB_MOVE = 1, SUB_MID = 2 };

// One problem: grid size, strip height, shifted wave number and the FP64 profile tables
// (all device pointers into one allocation owned by the problem handle).
struct ProbDev {
    int32_t n, B, c, L_lo, L_up, nsub;  // c: middle layer; L_lo/L_up: moving layers per front
    double ih2;                         // 1/h^2
    double2 kappa2;                     // (omega + i alpha)^2   (operator A_alpha)
    double2 omega2;                     // omega^2               (operator A)
    const double2 *s1n, *is1n, *s1h;    // x1: s, 1/s at ih (n); s at (i+1/2)h, i = 0..n (n+1)
    const double2 *s2n, *is2n, *s2h;    // x2 physical, same layout
    const double2 *mvn, *imvn, *mvh;    // moving strip: s, 1/s at local rows (B); halves (B+1)
    const double2 *mdn, *imdn, *mdh;    // middle strip: (2B-1); halves (2B)
    const double* ic2;                  // 1/c^2 on the grid (n*n)
};

// One subproblem strip for the factorisation kernel.
struct SubDev {
    int32_t prob;       // index into the ProbDev table
    int32_t kind;       // SubKind
    int32_t j0, dir;    // physical row (1-based) of local row 0, and +1/-1 going up the local rows
    int32_t cdir;       // column direction of the block LU: +1 (1 -> n) or -1 (n -> 1)
    int32_t jl;         // layer row of the strip (the row whose values leave the strip)
    int32_t jprev;      // layer row of the previous layer in the sweep (0: none)
    int32_t jnext;      // layer row of the next layer in the sweep (0: none)
    int64_t fac_off;    // offset of this strip's factor in its problem's store (complex elements)
    void* facp;         // absolute address of the strip's first stored column
    // The strip's x2 profile resolved on the host (no branch on the strip kind in device code):
    // local row r has s2 = rs2[rstep*r], 1/s2 = ris2[rstep*r], and s2 at the half rows below and
    // above it rlo[rstep*r], rhi[rstep*r].
    const double2 *rs2, *ris2, *rlo, *rhi;
    int32_t rstep;
    int32_t pad_;
};

// One sweep chain: a front of one problem and a group of right-hand sides.
struct ChainDev {
    int32_t prob;
    int32_t front;      // 0: upward front (F, B+1, ..., c-1); 1: downward front (E, n-B, ..., c+1)
    int32_t rhs0, nq;   // first right-hand side and count (<= lanes / padded rows)
    int32_t sys0;       // system index of the first right-hand side (batch order, problem-major)
    int32_t wrhs;       // segmented chains: waves per right-hand side (plain chains: unused)
    int64_t spill_off;  // offset of this chain's workspace (complex elements)
};

// True if one of the chain's systems is still active (the result is the same in every lane).
__device__ inline bool any_active(const int32_t* active, const ChainDev& ch) {
    int a = 0;
    for (int i = 0; i < ch.nq; ++i) a |= active[ch.sys0 + i];
    return a != 0;
}

// Per-problem vector pointers for one application of the sweep (or one matvec).
struct IoDev {
    const void* in;
    void* out;
    const void* fac;    // factor store of the problem (complex elements of the factor precision)
    const void* prop;   // segment propagators of the problem's front strips (segmented sweep), or nullptr
    const void* cmp;    // compressed blocks of the problem's moving strips (compressed chains), or nullptr
    const void* msp;    // split (bf16 hi / lo) copy of the F / E / moving strips' blocks (matrix-core chains), or nullptr
};

// Columns per segment of the segmented strip solves.
constexpr int SEG = 16;

// One propagator work item: Q consecutive segments (from seg0) of one front strip.
struct PropDev {
    int32_t prob;           // index into the ProbDev table
    int32_t cdir;           // column direction of the strip's block LU
    int32_t rstep;          // 1/s2 of local row r at ris2[rstep * r]
    int32_t seg0;
    const void* fac;        // first stored column of the strip
    const double2* ris2;
    void* out;              // the strip's propagators: [segment][row-major BS x BS block]
};

// One compression work item: one physical segment of one moving strip (k_compress).
struct CompDev {
    int32_t prob;           // index into the ProbDev table
    int32_t cdir;           // column direction of the strip's block LU
    int32_t rstep;          // 1/s2 of local row r at ris2[rstep * r]
    int32_t seg;            // physical segment (columns seg*SEG .. seg*SEG+SEG-1)
    const void* fac;        // first stored column of the strip
    const double2* ris2;
    void* out;              // the segment's compressed block
};

__host__ __device__ constexpr int packed_size(int bs) { return bs * (bs + 1) / 2; }

// Lanes per strip row group: a strip of BS rows occupies RP lanes (padded), Q = 64/RP groups per wave.
template <int BS> struct RowsOf {
    static constexpr int RP = BS <= 16 ? 16 : (BS <= 32 ? 32 : 64);
    static constexpr int Q = 64 / RP;
};

// One stored column of a strip factor: the packed upper triangle of Lambda_s^{-1} (PACK entries),
// then three coupling scalars (x1 coupling to the next step without the 1/s2 row factor;
// coupling of the layer row to the previous / next layer), padded to a multiple of 16 bytes.
constexpr int XCOL_E = 0, XCOL_APREV = 1, XCOL_ANEXT = 2;
template <class TF> __host__ __device__ constexpr int col_stride(int bs) {
    return sizeof(C2<TF>) == 8 ? ((packed_size(bs) + 3 + 1) & ~1) : packed_size(bs) + 3;
}
// index of (r, k), r <= k, in the row-major packed upper triangle of a bs x bs block
__host__ __device__ constexpr int packed_index(int bs, int r, int k) { return r * bs - (r * (r - 1)) / 2 + (k - r); }

// Profile of local row r of a strip described by a SubDev.
__device__ __forceinline__ void row_profile(const SubDev& S, int r, double2& s2, double2& is2, double2& s2lo,
                                            double2& s2hi) {
    const int o = S.rstep * r;
    s2 = gld(gptr(S.rs2 + o));
    is2 = gld(gptr(S.ris2 + o));
    s2lo = gld(gptr(S.rlo + o));
    s2hi = gld(gptr(S.rhi + o));
}

// Profile of local row r of a strip of a kind fixed at compile time: s2, 1/s2 at the row and s2 at
// the half rows below / above it.
__device__ __forceinline__ void strip_profile(const ProbDev& P, int kind, int j0, int dir, int r,
                                              double2& s2, double2& is2, double2& s2lo, double2& s2hi) {
    if (kind == SUB_PHYS) {
        int j = j0 + dir * r;
        s2 = P.s2n[j - 1];
        is2 = P.is2n[j - 1];
        if (dir > 0) { s2lo = P.s2h[j - 1]; s2hi = P.s2h[j]; }
        else         { s2lo = P.s2h[j];     s2hi = P.s2h[j - 1]; }
    } else if (kind == SUB_MOVE) {
        s2 = P.mvn[r]; is2 = P.imvn[r]; s2lo = P.mvh[r]; s2hi = P.mvh[r + 1];
    } else {
        s2 = P.mdn[r]; is2 = P.imdn[r]; s2lo = P.mdh[r]; s2hi = P.mdh[r + 1];
    }
}

}  // namespace hs
