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
//
// Every strip carries its own problem index and factor address, so one launch covers the strips of
// any number of problems of one strip height.
#include <float.h>

#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

// Maximum of a 32-bit key over each group of RP consecutive lanes; every lane gets its group's
// maximum.  Rows of 16 lanes reduce with DPP lane swaps (neighbours, pairs, half-row mirror, row
// mirror); wider groups combine the row results through scalar lane reads.  Must be called with all
// 64 lanes active.
template <int RP>
__device__ __forceinline__ uint32_t group_max(uint32_t key) {
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x141, 0xF, 0xF, false));  // row_half_mirror
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x140, 0xF, 0xF, false));  // row_mirror
    if (RP >= 32) {
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)key, 0);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)key, 16);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)key, 32);
        const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)key, 48);
        if (RP == 32) key = threadIdx.x < 32 ? max(a, b) : max(c, d);
        else key = max(max(a, b), max(c, d));
    }
    return key;
}

template <class TS, int BS>
__global__ __launch_bounds__(64) void k_factor(const ProbDev* __restrict__ probs, const SubDev* __restrict__ subs,
                                               int nsub, int* __restrict__ status) {
    constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q;
    constexpr int PACK = packed_size(BS);
    constexpr int STRIDE = col_stride<TS>(BS);
    // Gauss-Jordan result of this step, then (upper triangle, in place) the symmetrised inverse, which
    // the next step reads while building its Lambda
    __shared__ double2 sym_lds[Q][BS][BS + 1];
    __shared__ double2 prow[Q][BS];                // pivot row of the current elimination step
    __shared__ double2 e_lds[Q][BS];
    __shared__ double2 extra[Q][3];
    __shared__ uint16_t unpack[PACK];
    __shared__ uint64_t fac_lds[Q];               // strip factor address (0: group stores nothing)

    const int lane = threadIdx.x;
    const int g = lane / RP, r = lane % RP;
    const int sidx = blockIdx.x * Q + g;
    // A group owns a strip when its index is in range and the entry has a factor address (tables
    // of several problems are padded with address-less entries).  All groups of a wave must share
    // the column count n: group 0 (always in range) sets it; a group whose strip has another n
    // takes group 0's strip without storing it and reports the mismatch as status bit 2.
    SubDev S = subs[sidx < nsub ? sidx : nsub - 1];
    bool live = sidx < nsub && S.facp != nullptr;
    const int n = __builtin_amdgcn_readfirstlane(probs[S.prob].n);
    if (probs[S.prob].n != n) {
        if (live && (lane % RP) == 0) atomicOr(status + S.prob, 2);
        live = false;
        S = subs[blockIdx.x * Q];
    }
    const bool active = r < BS;
    const ProbDev& P = probs[S.prob];
    const double ih2 = P.ih2;
    const double2 kap2 = P.kappa2;

    for (int t = lane; t < PACK; t += 64) {
        int rr = 0, rem = t, len = BS;
        while (rem >= len) { rem -= len; --len; ++rr; }
        unpack[t] = (uint16_t)((rr << 8) | (rr + rem));
    }
    if (r == 0) fac_lds[g] = live ? (uint64_t)(uintptr_t)S.facp : 0;

    const int rc = active ? r : 0;
    double2 s2, is2, s2lo, s2hi;
    row_profile(S, rc, s2, is2, s2lo, s2hi);
    const int j = S.j0 + S.dir * rc;                          // physical row of local row r
    const HS_GLOBAL double* ic2row = gptr(P.ic2 + (int64_t)(j - 1) * n);
    const HS_GLOBAL double2* s1h = gptr(P.s1h);
    const HS_GLOBAL double2* is1n = gptr(P.is1n);
    const int cd = S.cdir;
    // x2 couplings of the layer row to the previous / next layer of the sweep, without the 1/s1 factor
    const double2 zero = make_double2(0.0, 0.0);
    const double2 cprev = S.jprev > 0 ? cscale<double>(gld(gptr(P.s2h + (S.jprev < S.jl ? S.jprev : S.jl))), ih2) : zero;
    const double2 cnext = S.jnext > 0 ? cscale<double>(gld(gptr(P.s2h + (S.jnext < S.jl ? S.jnext : S.jl))), ih2) : zero;

    // per-column coefficients, loaded one column ahead
    auto colof = [&](int s) __attribute__((always_inline)) { return cd > 0 ? s + 1 : n - s; };
    int col = colof(0);
    double2 is1 = gld(is1n + col - 1), s1l = gld(s1h + col - 1), s1r = gld(s1h + col);
    double ic2 = ic2row[col - 1];

    double2 slot[BS];
    int bad = 0;
    wave_sync();

    for (int s = 0; s < n; ++s) {
        const int coln = colof(s + 1 < n ? s + 1 : s);
        const double2 is1_n = gld(is1n + coln - 1), s1l_n = gld(s1h + coln - 1), s1r_n = gld(s1h + coln);
        const double ic2_n = ic2row[coln - 1];

        const double2 axl = cscale<double>(cmul<double>(s1l, is2), ih2);     // x1 coupling at col - 1/2
        const double2 axr = cscale<double>(cmul<double>(s1r, is2), ih2);     // at col + 1/2
        const double2 ayl = cscale<double>(cmul<double>(s2lo, is1), ih2);    // x2 coupling below
        const double2 ayh = cscale<double>(cmul<double>(s2hi, is1), ih2);    // above
        const double2 e = cd > 0 ? axl : axr;                                // to the previous step
        double2 d = cscale<double>(cmul<double>(cmul<double>(kap2, is1), is2), ic2);
        d = csub<double>(d, cadd<double>(cadd<double>(axl, axr), cadd<double>(ayl, ayh)));
        if (active) e_lds[g][r] = e;
        if (r == 0) {
            // x1 coupling between this step's column and the next step's (zero after the last step)
            extra[g][0] = s + 1 < n ? cscale<double>(cd > 0 ? s1r : s1l, ih2) : zero;
            extra[g][1] = cmul<double>(cprev, is1);
            extra[g][2] = cmul<double>(cnext, is1);
        }
        wave_sync();
        // row r of Lambda_s = D_s - E_s Lambda_{s-1}^{-1} E_s
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            double2 v = zero;
            if (k == r) v = d;
            else if (k == r - 1) v = ayl;
            else if (k == r + 1) v = ayh;
            if (s > 0) v = cfms<double>(cmul<double>(e, e_lds[g][k]), sym_lds[g][rc < k ? rc : k][rc < k ? k : rc], v);
            slot[k] = active ? v : zero;
        }

        // In-place Gauss-Jordan with partial pivoting inside each group of RP lanes.  The pivot of
        // step k is the unused row with the largest |re| + |im| in column k (ties: lowest row; the
        // key packs the FP32 magnitude above a validity bit and the inverted row index, so unused
        // rows with a zero or NaN entry still outrank used ones and a zero pivot is flagged).
        // Every lane applies the same update  row <- keep * row - f * pivot_row,  slot k <- -f:
        // other rows keep = 1, f = row[k] / a; the pivot row keep = 0, f = -1 / a, which leaves it
        // scaled by 1/a with 1/a in slot k.
        bool used = !active;
        int myrow = 0;
        int piv[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) {
            const float m = fabsf((float)slot[k].x) + fabsf((float)slot[k].y);
            const uint32_t mb = m >= 0.0f ? __float_as_uint(m) : 0u;
            uint32_t key = used ? 0u : (((mb >> 7) << 7) | 64u | (uint32_t)(63 - r));
            key = group_max<RP>(key);
            const int p = 63 - (int)(key & 63u);
            piv[k] = p;
            const bool me = r == p;
            if (me) {
#pragma unroll
                for (int q = 0; q < BS; ++q) prow[g][q] = slot[q];
            }
            wave_sync();
            const double2 a = prow[g][k];
            const double a2 = a.x * a.x + a.y * a.y;
            bad |= (a2 > 0.0 && a2 <= DBL_MAX) ? 0 : 1;
            const double ia2 = 1.0 / a2;
            const double2 ia = make_double2(a.x * ia2, -a.y * ia2);   // 1/a
            const double keep = me ? 0.0 : 1.0;
            const double2 fo = cmul<double>(slot[k], ia);
            const double2 f = make_double2(me ? -ia.x : fo.x, me ? -ia.y : fo.y);
#pragma unroll
            for (int q = 0; q < BS; ++q) {
                if (q == k) continue;
                slot[q] = cfms<double>(f, prow[g][q], make_double2(slot[q].x * keep, slot[q].y * keep));
            }
            slot[k] = make_double2(-f.x, -f.y);
            myrow = me ? k : myrow;
            used = used || me;
            wave_sync();
        }
        // lane p_k holds row k of the inverse: slot[q] = Inv[k][p_q] (the previous inverse has been read)
        if (active) {
#pragma unroll
            for (int q = 0; q < BS; ++q) sym_lds[g][myrow][piv[q]] = slot[q];
        }
        wave_sync();
        // symmetrise into the upper triangle: lane r writes only (r, k >= r) and reads (k, r) below the
        // diagonal, which no lane writes
        if (active) {
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                if (k < r) continue;
                const double2 x = sym_lds[g][r][k], y = sym_lds[g][k][r];
                sym_lds[g][r][k] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y + y.y));
            }
        }
        wave_sync();
        for (int t = lane; t < Q * STRIDE; t += 64) {
            const int gg = t / STRIDE, tt = t - gg * STRIDE;
            const uint64_t fa = fac_lds[gg];
            if (fa == 0) continue;
            HS_GLOBAL C2<TS>* fp = (HS_GLOBAL C2<TS>*)(uintptr_t)fa;
            // both LDS reads at valid indices, then a value select (no pointer select)
            const int u = unpack[tt < PACK ? tt : 0];
            const double2 vs = sym_lds[gg][u >> 8][u & 0xff];
            const double2 ve = extra[gg][(tt >= PACK && tt < PACK + 3) ? tt - PACK : 0];
            const bool is_s = tt < PACK, is_e = !is_s && tt < PACK + 3;
            const double2 v = make_double2(is_s ? vs.x : (is_e ? ve.x : 0.0), is_s ? vs.y : (is_e ? ve.y : 0.0));
            gst(fp + (int64_t)s * STRIDE + tt, ccast<TS, double>(v));
        }
        wave_sync();
        is1 = is1_n; s1l = s1l_n; s1r = s1r_n; ic2 = ic2_n;
    }
    if (bad && live && active) atomicOr(status + S.prob, 1);
}

template <class TS>
static bool dispatch_factor(int bs, const ProbDev* probs, const SubDev* subs, int nsub, int* status, hipStream_t s) {
    switch (bs) {
#define HS_CASE(BSV)                                                                                   \
    case BSV: {                                                                                        \
        dim3 g((nsub + RowsOf<BSV>::Q - 1) / RowsOf<BSV>::Q), b(64);                                  \
        hipLaunchKernelGGL((k_factor<TS, BSV>), g, b, 0, s, probs, subs, nsub, status);               \
        return true;                                                                                   \
    }
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17) HS_CASE(25) HS_CASE(33)
#undef HS_CASE
        default: return false;
    }
}

bool launch_factor(int bs, int prec, const ProbDev* probs, const SubDev* subs, int nsub, int* status, hipStream_t s) {
    if (nsub <= 0) return true;
    return prec == 0 ? dispatch_factor<double>(bs, probs, subs, nsub, status, s)
                     : dispatch_factor<float>(bs, probs, subs, nsub, status, s);
}

}  // namespace hs
