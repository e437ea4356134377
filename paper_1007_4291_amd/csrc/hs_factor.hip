// a2: block LU of every moving-PML strip (Section 2.2, Algorithm 3).
//
// A strip of BS rows, in the x2-first ordering, is block tridiagonal over the n columns:
//   H = tridiag(E_i, D_i, E_{i+1}),  D_i complex symmetric tridiagonal (BS x BS),
//   E_i = diag(e_i) the x1 couplings between columns i-1 and i.
// The block LU runs along the strip's column direction (left to right, or right to left for every
// other layer of a front, so that consecutive layers can be swept in lockstep):
//   Lambda_0 = D_col(0),  Lambda_s = D_col(s) - E_s Lambda_{s-1}^{-1} E_s.
// Each Lambda_s is inverted in FP64 by in-place Gauss-Jordan elimination with partial pivoting,
// one lane per row, RP lanes per strip (64/RP strips per wave).  The complex-symmetric inverse is
// symmetrised and stored packed (upper triangle, row-major) in the storage precision, followed by
// three coupling scalars per column: the x1 coupling to the next step's column (without the row
// factor 1/s2), and the couplings A_{j,j'} of the layer row to the previous and next layers of the
// sweep at this column.
#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

template <class TS, int BS>
__global__ __launch_bounds__(64) void k_factor(const ProbDev* __restrict__ prob, const SubDev* __restrict__ subs, int nsub,
                                               C2<TS>* __restrict__ fac, int* __restrict__ status) {
    constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q;
    constexpr int PACK = packed_size(BS);
    constexpr int STRIDE = col_stride<TS>(BS);
    __shared__ double2 inv_lds[Q][BS][BS + 1];
    __shared__ double2 sym_lds[Q][BS][BS + 1];
    __shared__ double2 prow[Q][BS];
    __shared__ double2 e_lds[Q][BS];
    __shared__ double2 extra[Q][3];
    __shared__ uint16_t unpack[PACK];
    __shared__ int64_t off_lds[Q];
    __shared__ int ok_lds[Q];

    const int lane = threadIdx.x;
    const int g = lane / RP, r = lane % RP;
    const int sidx = blockIdx.x * Q + g;
    const bool store_ok = sidx < nsub;
    const SubDev S = subs[store_ok ? sidx : nsub - 1];
    const bool active = r < BS;
    const ProbDev& P = prob[S.prob];
    const int n = P.n;
    const double ih2 = P.ih2;
    const double2 kap2 = P.kappa2;

    for (int t = lane; t < PACK; t += 64) {
        int rr = 0, rem = t, len = BS;
        while (rem >= len) { rem -= len; --len; ++rr; }
        unpack[t] = (uint16_t)((rr << 8) | (rr + rem));
    }
    if (r == 0) { off_lds[g] = S.fac_off; ok_lds[g] = store_ok ? 1 : 0; }

    const int rc = active ? r : 0;
    double2 s2, is2, s2lo, s2hi;
    row_profile(S, rc, s2, is2, s2lo, s2hi);
    const int j = S.j0 + S.dir * rc;                         // physical row of local row r
    const double* __restrict__ ic2row = P.ic2 + (int64_t)(j - 1) * n;
    const int cd = S.cdir;

    double2 slot[BS];
    int bad = 0;
    __syncthreads();

    for (int s = 0; s < n; ++s) {
        const int col = cd > 0 ? s + 1 : n - s;
        const double2 is1 = P.is1n[col - 1];
        const double2 axl = cscale<double>(cmul<double>(P.s1h[col - 1], is2), ih2);   // x1 coupling at col - 1/2
        const double2 axr = cscale<double>(cmul<double>(P.s1h[col], is2), ih2);       // at col + 1/2
        const double2 ayl = cscale<double>(cmul<double>(s2lo, is1), ih2);             // x2 coupling below
        const double2 ayh = cscale<double>(cmul<double>(s2hi, is1), ih2);             // above
        const double2 e = cd > 0 ? axl : axr;                                         // to the previous step
        double2 d = cscale<double>(cmul<double>(cmul<double>(kap2, is1), is2), ic2row[col - 1]);
        d = csub<double>(d, cadd<double>(cadd<double>(axl, axr), cadd<double>(ayl, ayh)));
        if (active) e_lds[g][r] = e;
        if (r == 0) {
            // x1 coupling between this step's column and the next step's (zero after the last step)
            const double2 es = cscale<double>(P.s1h[cd > 0 ? col : col - 1], ih2);
            extra[g][0] = s + 1 < n ? es : make_double2(0.0, 0.0);
            const double2 a1 = cscale<double>(is1, ih2);
            extra[g][1] = S.jprev > 0 ? cmul<double>(P.s2h[S.jprev < S.jl ? S.jprev : S.jl], a1) : make_double2(0.0, 0.0);
            extra[g][2] = S.jnext > 0 ? cmul<double>(P.s2h[S.jnext < S.jl ? S.jnext : S.jl], a1) : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            double2 v = make_double2(0.0, 0.0);
            if (k == r) v = d;
            else if (k == r - 1) v = ayl;
            else if (k == r + 1) v = ayh;
            if (s > 0 && active) v = cfms<double>(cmul<double>(e, e_lds[g][k]), sym_lds[g][r][k], v);   // - e_r e_k Lambda^{-1}_{rk}
            slot[k] = active ? v : make_double2(0.0, 0.0);
        }

        // in-place Gauss-Jordan with partial pivoting inside each group of RP lanes: after step k the
        // slot k of the pivot row's lane holds the right-hand column of that row (identity column p_k)
        bool used = !active;
        int myrow = 0;
        int piv[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            // unused rows compete with v >= 0 (a NaN magnitude counts as 0), so the pivot is always an
            // unused row of the group; a zero pivot is flagged below
            double v = cabs2<double>(slot[k]);
            if (!(v >= 0.0)) v = 0.0;
            if (used) v = -1.0;
            int idx = r;
#pragma unroll
            for (int off = RP / 2; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(v, off, RP);
                const int oi = __shfl_xor(idx, off, RP);
                if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
            }
            const int p = idx;
            if (!(v > 0.0) || !isfinite(v)) bad = 1;
            piv[k] = p;
            if (r == p) {
                const double2 ip = cinv<double>(slot[k]);
#pragma unroll
                for (int q = 0; q < BS; ++q) {
                    slot[q] = (q == k) ? ip : cmul<double>(slot[q], ip);
                    prow[g][q] = slot[q];
                }
                used = true;
                myrow = k;
            }
            __syncthreads();
            if (r != p && active) {
                const double2 f = slot[k];
#pragma unroll
                for (int q = 0; q < BS; ++q)
                    slot[q] = (q == k) ? cscale<double>(cmul<double>(f, prow[g][k]), -1.0) : cfms<double>(f, prow[g][q], slot[q]);
            }
            __syncthreads();
        }
        // lane p_k holds row k of the inverse: slot[q] = Inv[k][p_q]
        if (active) {
#pragma unroll
            for (int q = 0; q < BS; ++q) inv_lds[g][myrow][piv[q]] = slot[q];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                const double2 a = inv_lds[g][r][k], b = inv_lds[g][k][r];
                sym_lds[g][r][k] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
            }
        }
        __syncthreads();
        for (int t = lane; t < Q * STRIDE; t += 64) {
            const int gg = t / STRIDE, tt = t - gg * STRIDE;
            if (!ok_lds[gg]) continue;
            double2 v = make_double2(0.0, 0.0);
            if (tt < PACK) { const int rr = unpack[tt] >> 8, kk = unpack[tt] & 0xff; v = sym_lds[gg][rr][kk]; }
            else if (tt < PACK + 3) v = extra[gg][tt - PACK];
            fac[off_lds[gg] + (int64_t)s * STRIDE + tt] = ccast<TS, double>(v);
        }
        __syncthreads();
    }
    if (bad && store_ok && active) atomicOr(status, 1);
}

template <class TS>
static bool dispatch_factor(int bs, const ProbDev* prob, const SubDev* subs, int nsub, void* fac, int* status,
                            hipStream_t s) {
    C2<TS>* f = (C2<TS>*)fac;
    switch (bs) {
#define HS_CASE(BSV)                                                                                   \
    case BSV: {                                                                                        \
        dim3 g((nsub + RowsOf<BSV>::Q - 1) / RowsOf<BSV>::Q), b(64);                                  \
        hipLaunchKernelGGL((k_factor<TS, BSV>), g, b, 0, s, prob, subs, nsub, f, status);             \
        return true;                                                                                   \
    }
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
