// a3 / a4: application of the approximate sweeping LDL^t (Algorithm 4, two fronts + middle layer).
//
// One wavefront runs one chain (a front of one problem) for a group of right-hand sides.  Lane
// (q, r) = lane / RP, lane % RP owns row r of the strip for right-hand side q.  Each strip solve is
// the block LU solve over the n columns:
//   forward   w_i = Lambda_i^{-1} z_i,  z_{i+1} = g_{i+1} - e_{i+1} w_i     (w kept in a workspace)
//   backward  x_n = w_n,  x_i = w_i - Lambda_i^{-1} (e_{i+1} x_{i+1})
// The block-vector products exchange z through LDS; Lambda_i^{-1} rows are gathered from the
// packed symmetric store one column ahead of their use.
#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

template <int BS> struct PadRows { static constexpr int v = BS <= 16 ? 16 : (BS <= 32 ? 32 : 64); };

// Row r of the packed symmetric block at `col` (BS entries, zero for padding lanes).
template <class T, class TF, int BS>
__device__ __forceinline__ void load_row(const C2<TF>* __restrict__ col, int r, bool rowok, C2<T> (&L)[BS]) {
    r = rowok ? r : 0;
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int idx = (k >= r) ? (r * BS - (r * (r - 1)) / 2 + (k - r)) : (k * BS - (k * (k - 1)) / 2 + (r - k));
        L[k] = rowok ? ccast<T, TF>(col[idx]) : mk<T>(0, 0);
    }
}

// Block LU solve of one strip for the lane's (row, rhs); loadg(i) gives g at column i (1-based)
// for this lane, storex(i, x) receives the solution.  is2: 1/s2 of the lane's row.
template <class T, class TF, int BS, int RP, class LoadG, class StoreX>
__device__ __forceinline__ void strip_solve(const ProbDev& P, const C2<TF>* __restrict__ fac, double2 is2,
                                            C2<T>* __restrict__ spill, C2<T> (*zx)[64 / RP][RP],
                                            LoadG loadg, StoreX storex) {
    constexpr int PACK = packed_size(BS);
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const bool rowok = r < BS;
    const int n = P.n;
    const double ih2 = P.ih2;
    const double2 is2h = cscale<double>(is2, ih2);

    C2<T> Lc[BS], Ln[BS];
    load_row<T, TF, BS>(fac, r, rowok, Lc);
    C2<T> z = loadg(1);
    C2<T> w = mk<T>(0, 0);
    int buf = 0;
    for (int i = 1; i <= n; ++i) {
        if (i < n) load_row<T, TF, BS>(fac + (int64_t)i * PACK, r, rowok, Ln);
        zx[buf][q][r] = z;
        __syncthreads();
        C2<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int k = 0; k < BS; ++k) acc = cfma<T>(Lc[k], zx[buf][q][k], acc);
        w = acc;
        spill[(int64_t)(i - 1) * 64 + lane] = w;
        if (i < n) {
            const C2<T> e = ccast<T, double>(cmul<double>(P.s1h[i], is2h));     // coupling of columns i, i+1
            z = cfms<T>(e, w, loadg(i + 1));
#pragma unroll
            for (int k = 0; k < BS; ++k) Lc[k] = Ln[k];
        }
        buf ^= 1;
    }
    C2<T> x = w;
    storex(n, x);
    if (n > 1) load_row<T, TF, BS>(fac + (int64_t)(n - 2) * PACK, r, rowok, Lc);
    for (int i = n - 1; i >= 1; --i) {
        if (i > 1) load_row<T, TF, BS>(fac + (int64_t)(i - 2) * PACK, r, rowok, Ln);
        const C2<T> e = ccast<T, double>(cmul<double>(P.s1h[i], is2h));
        zx[buf][q][r] = cmul<T>(e, x);
        __syncthreads();
        C2<T> acc = spill[(int64_t)(i - 1) * 64 + lane];
#pragma unroll
        for (int k = 0; k < BS; ++k) acc = cfms<T>(Lc[k], zx[buf][q][k], acc);
        x = acc;
        storex(i, x);
        if (i > 1) {
#pragma unroll
            for (int k = 0; k < BS; ++k) Lc[k] = Ln[k];
        }
        buf ^= 1;
    }
}

template <class T> __device__ __forceinline__ C2<T> ld(const double2* p) { return ccast<T, double>(*p); }
template <class T> __device__ __forceinline__ C2<T> ld(const float2* p) { return ccast<T, float>(*p); }
template <class TO, class T> __device__ __forceinline__ TO cvt_out(C2<T> v);
template <> __device__ __forceinline__ double2 cvt_out<double2, double>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 cvt_out<double2, float>(float2 v) { return make_double2(v.x, v.y); }
template <> __device__ __forceinline__ float2 cvt_out<float2, float>(float2 v) { return v; }
template <> __device__ __forceinline__ float2 cvt_out<float2, double>(double2 v) { return make_float2((float)v.x, (float)v.y); }

// Coupling A_{j+1,j} at column i: (s2/s1)/h^2 at (ih, (j+1/2)h), j = the lower of the two rows.
__device__ __forceinline__ double2 row_coupling(const ProbDev& P, int jlo, int i) {
    return cscale<double>(cmul<double>(P.s2h[jlo], P.is1n[i - 1]), P.ih2);
}

template <class T, class TF, class TI, class TO, int BS>
__global__ __launch_bounds__(64) void k_chain(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                              const IoDev* __restrict__ io, IoDev io_val, int phase,
                                              C2<T>* __restrict__ spill_base) {
    constexpr int RP = PadRows<BS>::v;
    constexpr int Q = 64 / RP;
    constexpr int PACK = packed_size(BS);
    __shared__ C2<T> zx[2][Q][RP];
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const ChainDev ch = chains[blockIdx.x];
    const ProbDev& P = probs[ch.prob];
    const IoDev D = io ? io[ch.prob] : io_val;
    const int n = P.n, B = BS;
    const int64_t N = (int64_t)n * n;
    const bool qok = q < ch.nq;
    const bool act = qok && r < BS;
    const bool slot = act && r == B - 1;
    const int rhs = ch.rhs0 + (qok ? q : 0);
    const TI* __restrict__ fin = (const TI*)D.in + rhs * N;
    TO* __restrict__ y = (TO*)D.out + rhs * N;
    const C2<TF>* __restrict__ fac = (const C2<TF>*)D.fac;
    C2<T>* __restrict__ spill = spill_base + ch.spill_off;
    const int dir = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? B : n + 1 - B;
    const int L = ch.front == 0 ? P.L_lo : P.L_up;
    const int sub0 = ch.front == 0 ? 0 : P.L_lo + 1;
    const int64_t fstride = (int64_t)n * PACK;
    const int rr = r < BS ? r : 0;

    auto strip = [&](int t, auto loadg, auto storex) {
        const int jl = jF + dir * t;
        const int j0 = jl - dir * (B - 1);
        double2 s2, is2, s2lo, s2hi;
        strip_profile(P, t == 0 ? SUB_PHYS : SUB_MOVE, j0, dir, rr, s2, is2, s2lo, s2hi);
        strip_solve<T, TF, BS, RP>(P, fac + (int64_t)(sub0 + t) * fstride, is2, spill, zx, loadg, storex);
    };

    if (phase == 0) {
        // front block: all rows in, all rows out
        {
            const int jrow = jF - dir * (B - 1 - rr);
            const TI* gin = fin + (int64_t)(jrow - 1) * n;
            TO* xo = y + (int64_t)(jrow - 1) * n;
            strip(0, [&](int i) { return act ? ld<T>(gin + i - 1) : mk<T>(0, 0); },
                  [&](int i, C2<T> x) { if (act) xo[i - 1] = cvt_out<TO, T>(x); });
        }
        for (int t = 1; t <= L; ++t) {
            const int jl = jF + dir * t, jp = jl - dir, jlo = jl < jp ? jl : jp;
            const TI* gin = fin + (int64_t)(jl - 1) * n;
            const TO* yp = y + (int64_t)(jp - 1) * n;
            TO* xo = y + (int64_t)(jl - 1) * n;
            strip(t,
                  [&](int i) {
                      if (!slot) return mk<T>(0, 0);
                      const double2 a = row_coupling(P, jlo, i);
                      return ccast<T, double>(cfms<double>(a, ld<double>(yp + i - 1), ld<double>(gin + i - 1)));
                  },
                  [&](int i, C2<T> x) { if (slot) xo[i - 1] = cvt_out<TO, T>(x); });
        }
    } else {
        for (int t = L; t >= 0; --t) {
            const int jl = jF + dir * t, jn = jl + dir, jlo = jl < jn ? jl : jn;
            const TO* yn = y + (int64_t)(jn - 1) * n;
            auto loadg = [&](int i) {
                if (!slot) return mk<T>(0, 0);
                return ccast<T, double>(cmul<double>(row_coupling(P, jlo, i), ld<double>(yn + i - 1)));
            };
            if (t > 0) {
                TO* xo = y + (int64_t)(jl - 1) * n;
                strip(t, loadg, [&](int i, C2<T> x) {
                    if (slot) xo[i - 1] = cvt_out<TO, T>(csub<T>(ld<T>(xo + i - 1), x));
                });
            } else {
                const int jrow = jF - dir * (B - 1 - rr);
                TO* xo = y + (int64_t)(jrow - 1) * n;
                strip(0, loadg, [&](int i, C2<T> x) {
                    if (act) xo[i - 1] = cvt_out<TO, T>(csub<T>(ld<T>(xo + i - 1), x));
                });
            }
        }
    }
}

// Middle layer c: strip of 2B-1 rows damped on both sides; input u_c updated by both fronts.
template <class T, class TF, class TI, class TO, int BSM>
__global__ __launch_bounds__(64) void k_middle(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ mids,
                                               const IoDev* __restrict__ io, IoDev io_val, C2<T>* __restrict__ spill_base) {
    constexpr int RP = PadRows<BSM>::v;
    constexpr int Q = 64 / RP;
    __shared__ C2<T> zx[2][Q][RP];
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const ChainDev ch = mids[blockIdx.x];
    const ProbDev& P = probs[ch.prob];
    const IoDev D = io ? io[ch.prob] : io_val;
    const int n = P.n, B = P.B, c = P.c;
    const int64_t N = (int64_t)n * n;
    const bool qok = q < ch.nq;
    const bool slot = qok && r == B - 1;
    const int rhs = ch.rhs0 + (qok ? q : 0);
    const TI* __restrict__ gin = (const TI*)D.in + rhs * N + (int64_t)(c - 1) * n;
    TO* __restrict__ y = (TO*)D.out + rhs * N;
    const TO* ylo = y + (int64_t)(c - 2) * n;
    const TO* yhi = y + (int64_t)c * n;
    TO* xo = y + (int64_t)(c - 1) * n;
    const int64_t moff = (int64_t)(P.nsub - 1) * n * packed_size(B);
    const C2<TF>* __restrict__ fac = (const C2<TF>*)D.fac + moff;
    double2 s2, is2, s2lo, s2hi;
    strip_profile(P, SUB_MID, c - B + 1, 1, r < BSM ? r : 0, s2, is2, s2lo, s2hi);
    strip_solve<T, TF, BSM, RP>(P, fac, is2, spill_base + ch.spill_off, zx,
        [&](int i) {
            if (!slot) return mk<T>(0, 0);
            double2 g = ld<double>(gin + i - 1);
            g = cfms<double>(row_coupling(P, c - 1, i), ld<double>(ylo + i - 1), g);
            g = cfms<double>(row_coupling(P, c, i), ld<double>(yhi + i - 1), g);
            return ccast<T, double>(g);
        },
        [&](int i, C2<T> x) { if (slot) xo[i - 1] = cvt_out<TO, T>(x); });
}

// Test hook: one strip, every row in and out; vectors complex128 [nrhs][BS][n].
template <class T, class TF, int BS>
__global__ __launch_bounds__(64) void k_subsolve(const ProbDev* __restrict__ prob, const C2<TF>* __restrict__ fac,
                                                 int kind, int j0, int dir, const double2* __restrict__ g,
                                                 double2* __restrict__ x, int nrhs, C2<T>* __restrict__ spill) {
    constexpr int RP = PadRows<BS>::v;
    constexpr int Q = 64 / RP;
    __shared__ C2<T> zx[2][Q][RP];
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const ProbDev& P = *prob;
    const int n = P.n;
    const int rhs = blockIdx.x * Q + q;
    const bool act = rhs < nrhs && r < BS;
    const int64_t off = ((int64_t)(act ? rhs : 0) * BS + (r < BS ? r : 0)) * n;
    double2 s2, is2, s2lo, s2hi;
    strip_profile(P, kind, j0, dir, r < BS ? r : 0, s2, is2, s2lo, s2hi);
    strip_solve<T, TF, BS, RP>(P, fac, is2, spill + (int64_t)blockIdx.x * n * 64, zx,
        [&](int i) { return act ? ccast<T, double>(g[off + i - 1]) : mk<T>(0, 0); },
        [&](int i, C2<T> v) { if (act) x[off + i - 1] = cvt_out<double2, T>(v); });
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
template <class T, class TF, class TI, class TO>
static bool chains_typed(int B, int phase, const ProbDev* probs, const ChainDev* chains, int nch, const IoDev* io,
                         IoDev iov, void* spill, hipStream_t s) {
    dim3 g(nch), b(64);
    C2<T>* sp = (C2<T>*)spill;
    switch (B) {
#define HS_CASE(BV) case BV: hipLaunchKernelGGL((k_chain<T, TF, TI, TO, BV>), g, b, 0, s, probs, chains, io, iov, phase, sp); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17)
#undef HS_CASE
        default: return false;
    }
}

template <class T, class TF, class TI, class TO>
static bool middle_typed(int B, const ProbDev* probs, const ChainDev* mids, int nm, const IoDev* io, IoDev iov,
                         void* spill, hipStream_t s) {
    dim3 g(nm), b(64);
    C2<T>* sp = (C2<T>*)spill;
    switch (2 * B - 1) {
#define HS_CASE(BV) case BV: hipLaunchKernelGGL((k_middle<T, TF, TI, TO, BV>), g, b, 0, s, probs, mids, io, iov, sp); return true;
        HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17) HS_CASE(25) HS_CASE(33)
#undef HS_CASE
        default: return false;
    }
}

bool launch_chains(int B, int prec, int in_prec, int out_prec, int phase, const ProbDev* probs,
                   const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill, hipStream_t s) {
    if (nchains <= 0) return true;
    if (prec == 0) {
        if (in_prec == 0 && out_prec == 0) return chains_typed<double, double, double2, double2>(B, phase, probs, chains, nchains, io, io_val, spill, s);
        return false;
    }
    if (in_prec == 0 && out_prec == 1) return chains_typed<float, float, double2, float2>(B, phase, probs, chains, nchains, io, io_val, spill, s);
    if (in_prec == 1 && out_prec == 1) return chains_typed<float, float, float2, float2>(B, phase, probs, chains, nchains, io, io_val, spill, s);
    if (in_prec == 0 && out_prec == 0) return chains_typed<float, float, double2, double2>(B, phase, probs, chains, nchains, io, io_val, spill, s);
    return false;
}

bool launch_middle(int B, int prec, int in_prec, int out_prec, const ProbDev* probs, const ChainDev* mids,
                   int nmids, const IoDev* io, IoDev io_val, void* spill, hipStream_t s) {
    if (nmids <= 0) return true;
    if (prec == 0) {
        if (in_prec == 0 && out_prec == 0) return middle_typed<double, double, double2, double2>(B, probs, mids, nmids, io, io_val, spill, s);
        return false;
    }
    if (in_prec == 0 && out_prec == 1) return middle_typed<float, float, double2, float2>(B, probs, mids, nmids, io, io_val, spill, s);
    if (in_prec == 1 && out_prec == 1) return middle_typed<float, float, float2, float2>(B, probs, mids, nmids, io, io_val, spill, s);
    if (in_prec == 0 && out_prec == 0) return middle_typed<float, float, double2, double2>(B, probs, mids, nmids, io, io_val, spill, s);
    return false;
}

int chain_padded_rows(int B) { return B <= 16 ? 16 : (B <= 32 ? 32 : 64); }
int chain_rhs_per_wave(int B) { return 64 / chain_padded_rows(B); }
int middle_rhs_per_wave(int B) { return 64 / chain_padded_rows(2 * B - 1); }

template <class T, class TF>
static bool subsolve_typed(int bs, const ProbDev* prob, const void* fac, int kind, int j0, int dir, const void* g,
                           void* x, int nrhs, void* spill, hipStream_t s) {
    const int Q = 64 / chain_padded_rows(bs);
    dim3 gr((nrhs + Q - 1) / Q), b(64);
    switch (bs) {
#define HS_CASE(BV) case BV: hipLaunchKernelGGL((k_subsolve<T, TF, BV>), gr, b, 0, s, prob, (const C2<TF>*)fac, kind, j0, dir, \
                                                (const double2*)g, (double2*)x, nrhs, (C2<T>*)spill); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17) HS_CASE(25) HS_CASE(33)
#undef HS_CASE
        default: return false;
    }
}

bool launch_subsolve(int bs, int prec, const ProbDev* prob, const void* fac, int kind, int j0, int dir,
                     const void* g, void* x, int nrhs, void* spill, hipStream_t s) {
    return prec == 0 ? subsolve_typed<double, double>(bs, prob, fac, kind, j0, dir, g, x, nrhs, spill, s)
                     : subsolve_typed<float, float>(bs, prob, fac, kind, j0, dir, g, x, nrhs, spill, s);
}

}  // namespace hs
