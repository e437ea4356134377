// a2: block LU of every moving-PML strip (Section 2.2, Algorithm 3), one wavefront per strip.
//
// A strip of BS rows, in the x2-first ordering, is block tridiagonal over the n columns:
//   H = tridiag(E_i, D_i, E_{i+1}),  D_i complex symmetric tridiagonal (BS x BS),
//   E_i = diag(e_i) the x1 couplings between columns i-1 and i.
// Its block LU recurrence is Lambda_1 = D_1, Lambda_i = D_i - E_i Lambda_{i-1}^{-1} E_i.  Each
// Lambda_i is inverted in FP64 by in-place Gauss-Jordan elimination with partial pivoting, lane r
// holding row r; the complex-symmetric inverse is symmetrised, kept in registers for the next
// column and written packed (upper triangle, row-major) in the storage precision.
#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

template <class TS, int BS>
__global__ __launch_bounds__(64) void k_factor(const ProbDev* __restrict__ prob, const SubDev* __restrict__ subs,
                                               C2<TS>* __restrict__ fac, int* __restrict__ status) {
    constexpr int PACK = packed_size(BS);
    __shared__ double2 inv_lds[BS][BS + 1];
    __shared__ double2 sym_lds[BS][BS + 1];
    __shared__ double2 prow[BS];
    __shared__ double2 e_lds[BS];
    __shared__ uint16_t unpack[PACK];

    const int lane = threadIdx.x;
    const bool active = lane < BS;
    const SubDev S = subs[blockIdx.x];
    const ProbDev& P = prob[S.prob];
    const int n = P.n;
    const double ih2 = P.ih2;
    const double2 kap2 = P.kappa2;

    for (int t = lane; t < PACK; t += 64) {
        int rr = 0, rem = t, len = BS;
        while (rem >= len) { rem -= len; --len; ++rr; }
        unpack[t] = (uint16_t)((rr << 8) | (rr + rem));
    }

    const int r = active ? lane : 0;
    double2 s2, is2, s2lo, s2hi;
    strip_profile(P, S.kind, S.j0, S.dir, r, s2, is2, s2lo, s2hi);
    const int j = S.j0 + S.dir * r;                         // physical row of local row r
    const double* __restrict__ ic2row = P.ic2 + (int64_t)(j - 1) * n;
    C2<TS>* __restrict__ out = fac + S.fac_off;

    double2 prev[BS];
    double2 slot[BS];
#pragma unroll
    for (int k = 0; k < BS; ++k) prev[k] = make_double2(0.0, 0.0);
    int bad = 0;
    __syncthreads();

    for (int i = 1; i <= n; ++i) {
        const double2 is1 = P.is1n[i - 1];
        const double2 e = cscale<double>(cmul<double>(P.s1h[i - 1], is2), ih2);     // x1 coupling at i - 1/2
        const double2 axr = cscale<double>(cmul<double>(P.s1h[i], is2), ih2);       // at i + 1/2
        const double2 ayl = cscale<double>(cmul<double>(s2lo, is1), ih2);           // x2 coupling below
        const double2 ayh = cscale<double>(cmul<double>(s2hi, is1), ih2);           // above
        double2 d = cscale<double>(cmul<double>(cmul<double>(kap2, is1), is2), ic2row[i - 1]);
        d = csub<double>(d, cadd<double>(cadd<double>(e, axr), cadd<double>(ayl, ayh)));
        if (active) e_lds[lane] = e;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            double2 v = make_double2(0.0, 0.0);
            if (k == r) v = d;
            else if (k == r - 1) v = ayl;
            else if (k == r + 1) v = ayh;
            if (i > 1) v = cfms<double>(cmul<double>(e, e_lds[k]), prev[k], v);     // - e_r e_k Lambda^{-1}_{rk}
            slot[k] = active ? v : make_double2(0.0, 0.0);
        }

        // in-place Gauss-Jordan with partial pivoting: after step k the slot k of the pivot row's
        // lane holds the right-hand column of the pivot row (identity column p_k)
        bool used = !active;
        int myrow = 0;
        int piv_lane[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            // unused active lanes always compete with v >= 0 (a NaN magnitude counts as 0), so the
            // pivot is always an unused row of this strip; a zero pivot is flagged below
            double v = cabs2<double>(slot[k]);
            if (!(v >= 0.0)) v = 0.0;
            if (used) v = -1.0;
            int idx = lane;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                double ov = __shfl_xor(v, off);
                int oi = __shfl_xor(idx, off);
                if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
            }
            const int p = __builtin_amdgcn_readfirstlane(idx);
            if (!(v > 0.0) || !isfinite(v)) bad = 1;
            piv_lane[k] = p;
            if (lane == p) {
                const double2 ip = cinv<double>(slot[k]);
#pragma unroll
                for (int q = 0; q < BS; ++q) {
                    slot[q] = (q == k) ? ip : cmul<double>(slot[q], ip);
                    prow[q] = slot[q];
                }
                used = true;
                myrow = k;
            }
            __syncthreads();
            if (lane != p && active) {
                const double2 f = slot[k];
#pragma unroll
                for (int q = 0; q < BS; ++q)
                    slot[q] = (q == k) ? cscale<double>(cmul<double>(f, prow[k]), -1.0) : cfms<double>(f, prow[q], slot[q]);
            }
            __syncthreads();
        }
        // lane p_k holds row k of the inverse: slot[q] = Inv[k][p_q]
        if (active) {
#pragma unroll
            for (int q = 0; q < BS; ++q) inv_lds[myrow][piv_lane[q]] = slot[q];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                const double2 a = inv_lds[lane][k], b = inv_lds[k][lane];
                prev[k] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
                sym_lds[lane][k] = prev[k];
            }
        }
        __syncthreads();
        C2<TS>* __restrict__ col = out + (int64_t)(i - 1) * PACK;
        for (int t = lane; t < PACK; t += 64) {
            const int rr = unpack[t] >> 8, kk = unpack[t] & 0xff;
            col[t] = ccast<TS, double>(sym_lds[rr][kk]);
        }
        __syncthreads();
    }
    if (bad && lane == 0) atomicOr(status, 1);
}

template <class TS>
static bool dispatch_factor(int bs, const ProbDev* prob, const SubDev* subs, int nsub, void* fac, int* status,
                            hipStream_t s) {
    dim3 g(nsub), b(64);
    C2<TS>* f = (C2<TS>*)fac;
    switch (bs) {
#define HS_CASE(BSV) case BSV: hipLaunchKernelGGL((k_factor<TS, BSV>), g, b, 0, s, prob, subs, f, status); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17) HS_CASE(25) HS_CASE(33)
#undef HS_CASE
        default: return false;
    }
}

bool launch_factor(int bs, int prec, const ProbDev* prob, const SubDev* subs, int nsub, int n, void* fac,
                   int* status, hipStream_t s) {
    (void)n;
    if (nsub <= 0) return true;
    return prec == 0 ? dispatch_factor<double>(bs, prob, subs, nsub, fac, status, s)
                     : dispatch_factor<float>(bs, prob, subs, nsub, fac, status, s);
}

}  // namespace hs
