// a3 / a4: application of the approximate sweeping LDL^t (Algorithm 4, two fronts + middle layer).
//
// One wavefront runs one chain: the layers of one front of one problem, in the order of a phase
// (forward substitution: F, B+1, ..., c-1; backward substitution: c-1, ..., B+1, F; likewise for the
// downward front), for a group of right-hand sides.  Lane (q, r) = (lane / RP, lane % RP) owns row r
// of the strip for right-hand side q.  Each strip solve is the block LU solve along the strip's
// column direction (step s = 0..n-1):
//   forward   w_s = Lambda_s^{-1} z_s,   z_{s+1} = g_{s+1} - e_{s,s+1} w_s      (w kept in a workspace)
//   backward  x_{n-1} = w_{n-1},  x_s = w_s - Lambda_s^{-1} (e_{s,s+1} x_{s+1})
// Consecutive layers of a front are factored in opposite column directions, so the backward pass of
// layer t emits its layer-row values in exactly the column order in which the forward pass of layer
// t+1 consumes them: the two passes run in lockstep, one column ("tick") apart, two independent
// block-vector products per tick.  Factor columns, workspace values and inputs are prefetched D ticks
// ahead through a register ring and staged in LDS; the block-vector products exchange vectors in LDS.
#include "hs_sweep_util.h"

namespace hs {

template <class T, class TF, class TI, class TO, int BS, int MODE, int D, int KS>
__global__ __launch_bounds__(64) void k_sweep(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                              const IoDev* __restrict__ io, IoDev io_val, C2<T>* __restrict__ spill_base,
                                              const int32_t* __restrict__ active, SubArg sa) {
    using CT = C2<T>;
    using CF = C2<TF>;
    constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q;
    using CC = ColChunks<TF, BS>;
    constexpr int STRIDE = CC::STRIDE, N16 = CC::N16, NCH = CC::NCH;
    constexpr int PACK = packed_size(BS);
    // forward products of the last LAG steps, needed by the first backward steps before the
    // workspace copies written at the end of the previous pair can be prefetched
    constexpr int LAG = (D - 1) / 2 > 0 ? (D - 1) / 2 : 1;
    __shared__ chunk16 colb[N16];
    __shared__ chunk16 colf[2][N16];
    __shared__ CT xbx[Q][RP];
    __shared__ CT xfx[Q][RP];

    // lane = q * RP + r; with KS > 1 the KS groups q = KS*rq + kg share one right-hand side rq and
    // split each row-dot product over k = kg, kg + KS, ... (combined by cross-group shuffles)
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const int rq = q / KS, kg = q % KS;
    constexpr int KMAX = (BS + KS - 1) / KS;
    ChainDev ch{0, 0, 0, 0, 0, 0, 0};
    if (MODE != MODE_SUB) {
        ch = chains[blockIdx.x];
        if (active && !any_active(active, ch)) return;   // every right-hand side of the chain is frozen
    }
    const ProbDev& P = probs[ch.prob];
    const IoDev IO = io ? io[ch.prob] : io_val;
    // problem scalars, loaded once
    const int n = P.n, B = P.B, cmid = P.c, nsub = P.nsub;
    const int L = ch.front == 0 ? P.L_lo : P.L_up;
    const int sub0 = ch.front == 0 ? 0 : P.L_lo + 1;
    const int64_t N = (int64_t)n * n;
    constexpr int QR = Q / KS;                                    // right-hand sides per wave
    const int nq = MODE == MODE_SUB ? min(QR, sa.nrhs - (int)blockIdx.x * QR) : ch.nq;
    const bool qok = rq < nq;
    const bool rok = r < BS;
    const bool act = qok && rok;                                  // lane holds a row of a live system
    const bool own = act && kg == 0;                              // ... and writes it
    const bool slot = (MODE == MODE_SUB) ? false : (act && r == B - 1);
    const bool oslot = slot && kg == 0;
    const int rhs = (MODE == MODE_SUB ? (int)blockIdx.x * QR : ch.rhs0) + (qok ? rq : 0);
    const int rr = rok ? r : 0;
    const HS_GLOBAL TI* __restrict__ fin = gptr((const TI*)IO.in + rhs * N);
    HS_GLOBAL TO* __restrict__ y = gptr((TO*)IO.out + rhs * N);
    HS_GLOBAL C2<T>* __restrict__ spill = gptr(spill_base + (MODE == MODE_SUB ? (int64_t)blockIdx.x * chain_spill_elems(n) : ch.spill_off));
    // per-lane 16-byte slot after the workspace: the target of stores of ticks that have no output
    HS_GLOBAL char* const dummy = (HS_GLOBAL char*)(spill + (int64_t)2 * n * 64) + 16 * lane;
    const HS_GLOBAL char* const facbase = gptr(MODE == MODE_SUB ? (const char*)sa.fac : (const char*)IO.fac);
    const HS_GLOBAL double2* const sag = gptr(sa.g);
    HS_GLOBAL double2* const sax = gptr(sa.x);

    // the program: strips 0..m in processing order
    const int dirF = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? B : n + 1 - B;
    const int64_t bstride = (int64_t)n * col_stride<TF>(B);          // elements per B-row strip
    const int m = (MODE == MODE_FWD || MODE == MODE_BWD) ? L : 0;
    auto strip_t = [&](int i) __attribute__((always_inline)) { return MODE == MODE_FWD ? i : L - i; };
    auto strip_dir = [&](int i) __attribute__((always_inline)) -> int {   // also for the virtual strip m+1
        if (MODE == MODE_FWD || MODE == MODE_BWD) return (strip_t(i) & 1) ? -1 : 1;
        const int d0 = MODE == MODE_SUB ? sa.cdir : 1;
        return i == 0 ? d0 : -d0;
    };
    // first stored column of strip i (a valid address for every i in [0, m])
    auto strip_fac = [&](int i) __attribute__((always_inline)) -> const HS_GLOBAL char* {
        if (MODE == MODE_FWD || MODE == MODE_BWD) return facbase + sizeof(CF) * ((int64_t)(sub0 + strip_t(i)) * bstride);
        if (MODE == MODE_MID) return facbase + sizeof(CF) * ((int64_t)(nsub - 1) * bstride);
        return facbase;
    };
    auto strip_full = [&](int i) __attribute__((always_inline)) -> bool {
        if (MODE == MODE_FWD || MODE == MODE_BWD) return strip_t(i) == 0;
        return MODE == MODE_SUB;
    };
    // physical row of this lane (full strips) or of the layer row (others), 1-based
    auto strip_row = [&](int i, bool full) __attribute__((always_inline)) -> int {
        if (MODE == MODE_FWD || MODE == MODE_BWD) {
            const int jl = jF + dirF * strip_t(i);
            return full ? jl - dirF * (B - 1 - rr) : jl;
        }
        return cmid;
    };
    auto colof = [&](int d, int k) __attribute__((always_inline)) { return d > 0 ? k + 1 : n - k; };

    // 1/s2 of this lane's row: front blocks use the physical profile, moving layers the moving one
    CT is2_front = mk<T>(0, 0), is2_other = mk<T>(0, 0);
    {
        double2 s2, is2, lo, hi;
        if (MODE == MODE_FWD || MODE == MODE_BWD) {
            strip_profile(P, SUB_PHYS, jF - dirF * (B - 1), dirF, rr, s2, is2, lo, hi);
            is2_front = ccast<T, double>(is2);
            strip_profile(P, SUB_MOVE, 0, 1, rr, s2, is2, lo, hi);
            is2_other = ccast<T, double>(is2);
        } else if (MODE == MODE_MID) {
            strip_profile(P, SUB_MID, 0, 1, rr, s2, is2, lo, hi);
            is2_other = ccast<T, double>(is2);
        } else {
            is2_other = ccast<T, double>(gld(gptr(sa.ris2 + sa.rstep * rr)));
        }
    }
    auto strip_is2 = [&](int i) __attribute__((always_inline)) -> CT {
        if (MODE == MODE_FWD || MODE == MODE_BWD) return strip_t(i) == 0 ? is2_front : is2_other;
        return is2_other;
    };

    static_assert(D % 2 == 0, "the staging parity k & 1 must be a compile-time value");
    // register ring
    chunk16 rbk[D][NCH], rfk[D][NCH];
    CT rsp[D];
    double2 ra[D], rb2[D], rc[D];

    // A pair (strip i-1 backward, strip i forward) takes n + 1 ticks, padded to whole groups of D.
    const int TP = (n + 1 + D - 1) / D * D;
    const int G = TP / D;
    const int64_t colbytes = (int64_t)sizeof(CF) * STRIDE;

    // Prefetch cursor: group pg of pair pi, one group (D ticks) ahead of execution.  Loads are
    // unconditional: positions past the end are clamped to valid memory and their values are never
    // used.  Strip-dependent bases are recomputed only when the cursor enters a new pair.
    int pi = 0, pg = 0, pdir = 1;
    const HS_GLOBAL char* pfb = facbase;         // backward strip pi-1, column n-1 (stepping down)
    const HS_GLOBAL char* pff = facbase;         // forward strip pi, column 0 (stepping up)
    const HS_GLOBAL C2<T>* pspb = spill;         // workspace of strip pi-1, step n-1
    const HS_GLOBAL TI* pfrow = fin;             // MODE_FWD: input row of strip pi
    const HS_GLOBAL TO* pyrow = y;               // MODE_BWD: output row of strip pi-1
    auto pset = [&]() __attribute__((always_inline)) {
        const int pc = pi <= m + 1 ? pi : m + 1;
        const int ib = pc >= 1 ? pc - 1 : 0, ifw = pc <= m ? pc : m;
        pdir = strip_dir(pc);
        pfb = strip_fac(ib) + colbytes * (n - 1);
        pff = strip_fac(ifw);
        pspb = spill + (int64_t)(ib & 1) * n * 64 + (int64_t)(n - 1) * 64 + lane;
        if (MODE == MODE_FWD) pfrow = fin + (int64_t)(strip_row(ifw, strip_full(ifw)) - 1) * n;
        if (MODE == MODE_BWD) pyrow = y + (int64_t)(strip_row(ib, strip_full(ib)) - 1) * n;
    };
    pset();
    auto prefetch = [&](int u, chunk16 (&bk)[NCH], chunk16 (&fk)[NCH], CT& sp, double2& a0, double2& a1,
                        double2& a2) __attribute__((always_inline)) {
        const int pk = pg * D + u;
        const int k2 = pk < n ? pk : n - 1;
        const int col = pdir > 0 ? k2 + 1 : n - k2;
        const HS_GLOBAL chunk16* srcb = (const HS_GLOBAL chunk16*)(pfb - colbytes * k2);
        const HS_GLOBAL chunk16* srcf = (const HS_GLOBAL chunk16*)(pff + colbytes * k2);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int idx = c * 64 + lane < N16 ? c * 64 + lane : N16 - 1;
            bk[c] = srcb[idx];
            fk[c] = srcf[idx];
        }
        sp = gld(pspb - (int64_t)k2 * 64);
        if (MODE == MODE_FWD) {
            a0 = ld2(pfrow + col - 1);
        } else if (MODE == MODE_BWD) {
            a0 = ld2(y + (int64_t)(cmid - 1) * n + col - 1);
            a1 = ld2(pyrow + col - 1);
        } else if (MODE == MODE_MID) {
            a0 = ld2(fin + (int64_t)(cmid - 1) * n + col - 1);
            a1 = ld2(y + (int64_t)(cmid - 2) * n + col - 1);
            a2 = ld2(y + (int64_t)cmid * n + col - 1);
        } else {
            a0 = gld(sag + ((int64_t)rhs * BS + rr) * n + col - 1);
        }
    };
    auto prefetch_next_group = [&]() __attribute__((always_inline)) {
        if (++pg == G) { pg = 0; ++pi; pset(); }
    };

    // Lambda^{-1} row r of a staged column (packed upper triangle) times the exchange vector of group q:
    // element offsets of this lane's row entries k = kg + KS j are computed once
    int loff[KMAX];
#pragma unroll
    for (int jj = 0; jj < KMAX; ++jj) {
        const int k = kg + KS * jj < BS ? kg + KS * jj : BS - 1;
        loff[jj] = (k >= rr) ? (rr * BS - (rr * (rr - 1)) / 2 + (k - rr)) : (k * BS - (k * (k - 1)) / 2 + (rr - k));
    }
    auto rowdot = [&](const chunk16* colv, const CT (*xv)[RP]) __attribute__((always_inline)) -> CT {
        const CF* cf = (const CF*)colv;
        CT acc0 = mk<T>(0, 0), acc1 = mk<T>(0, 0);
#pragma unroll
        for (int jj = 0; jj < KMAX; ++jj) {
            const int k = kg + KS * jj;                   // k >= BS only in the last round of a k-split
            const CT l = ccast<T, TF>(cf[loff[jj]]);
            const CT xk = xv[q][KS == 1 ? jj : (k < BS ? k : 0)];
            const CT t = csel<T>(KS == 1 || k < BS, xk, mk<T>(0, 0));
            if (jj & 1) acc1 = cfma<T>(l, t, acc1);
            else acc0 = cfma<T>(l, t, acc0);
        }
        CT acc = cadd<T>(acc0, acc1);
        // sum of the KS partial products over the row groups of one right-hand side (lanes r + RP j):
        // a butterfly over the lane offsets RP, 2 RP, ..., RP * KS / 2
        if (RP <= 16 && RP * KS >= 32) { acc.x = xor_sum<16>(acc.x); acc.y = xor_sum<16>(acc.y); }
        if (RP <= 32 && RP * KS >= 64) { acc.x = xor_sum<32>(acc.x); acc.y = xor_sum<32>(acc.y); }
        return acc;
    };
    auto colscalar = [&](const chunk16* colv, int which) __attribute__((always_inline)) -> CT {
        return ccast<T, TF>(((const CF*)colv)[PACK + which]);
    };

    static_for<D>([&](auto UC) __attribute__((always_inline)) {
        constexpr int u = decltype(UC)::value;
        prefetch(u, rbk[u], rfk[u], rsp[u], ra[u], rb2[u], rc[u]);
    });
    prefetch_next_group();

    CT xcur = mk<T>(0, 0), z = mk<T>(0, 0), w = mk<T>(0, 0), wcarry = mk<T>(0, 0), ypart = mk<T>(0, 0);
    CT wlag[LAG], wsnap[LAG];
#pragma unroll
    for (int j = 0; j < LAG; ++j) { wlag[j] = mk<T>(0, 0); wsnap[j] = mk<T>(0, 0); }

    // Every tick issues the same sequence of global loads and stores (stores without output go to
    // the dummy slot), so the compiler's memory waits at each tick cover exactly the loads issued
    // D ticks earlier.
    for (int i = 0; i <= m + 1; ++i) {
        // pair i: backward pass of strip i-1 (i >= 1), forward pass of strip i (i <= m)
        const int ib = i >= 1 ? i - 1 : 0, ifw = i <= m ? i : m;
        const bool full_b = strip_full(ib), full_f = strip_full(ifw);
        const int row_b = strip_row(ib, full_b);
        const CT is2b = strip_is2(ib), is2f = strip_is2(ifw);
        const int cd = strip_dir(i);
        const bool pb = i >= 1, pf = i <= m;
        // layer output of this pair's backward pass: row base and whether this lane writes it
        bool wy;
        HS_GLOBAL TO* yrow;
        if (MODE == MODE_FWD || MODE == MODE_BWD) { wy = full_b ? own : oslot; yrow = y + (int64_t)(row_b - 1) * n; }
        else if (MODE == MODE_MID) { wy = oslot; yrow = y + (int64_t)(cmid - 1) * n; }
        else { wy = own; yrow = (HS_GLOBAL TO*)sax + ((int64_t)rhs * BS + r) * n; }
        wy = wy && pb;
        HS_GLOBAL CT* const spw = spill + (int64_t)(i & 1) * n * 64 + lane;   // forward products of strip i

        for (int kb = 0; kb < G; ++kb) {
            static_for<D>([&](auto UC) __attribute__((always_inline)) {
                constexpr int u = decltype(UC)::value;
                const int k = kb * D + u;
                const bool bon = k < n;                 // with pb: step n-1-k of strip i-1
                const bool fon = pf && k >= 1 && k <= n;
                const bool fin_on = pf && k < n;
                const int col = cd > 0 ? k + 1 : n - k;
                // stage the columns of this tick and the exchange vectors
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    // lanes past the column hold the clamped last chunk and rewrite it unchanged
                    const int idx = c * 64 + lane < N16 ? c * 64 + lane : N16 - 1;
                    colb[idx] = rbk[u][c];
                    colf[u & 1][idx] = rfk[u][c];
                }
                xbx[q][r] = cmul<T>(is2b, xcur);
                xfx[q][r] = z;
                wave_sync();
                // backward pass of strip i-1, step s = n-1-k
                CT ws = rsp[u];
#pragma unroll
                for (int j = 0; j < LAG; ++j) ws = csel<T>(k == j + 1, wsnap[j], ws);
                const CT xb = cfms<T>(colscalar(colb, XCOL_E), rowdot(colb, xbx), ws);
                // forward pass of strip i: product for step k-1
                const chunk16* cprev = colf[(u + 1) & 1];
                const CT wf = rowdot(cprev, xfx);
                // layer output of the backward pass
                const CT x = csel<T>(k == 0, wcarry, xb);
                const CT yval = MODE == MODE_BWD ? csub<T>(ccast<T, double>(rb2[u]), x) : x;
                gst((wy && bon) ? yrow + col - 1 : (HS_GLOBAL TO*)dummy, cvt_out<TO, T>(yval));
                if (pb && bon) {
                    xcur = x;
                    ypart = yval;
                }
                // forward product of step k-1 into the workspace
                gst(fon ? spw + (int64_t)(k - 1) * 64 : (HS_GLOBAL CT*)dummy, wf);
                if (fon) {
#pragma unroll
                    for (int j = LAG - 1; j >= 1; --j) wlag[j] = wlag[j - 1];
                    wlag[0] = w;
                    w = wf;
                    if (k == n) {
                        wcarry = w;
#pragma unroll
                        for (int j = 0; j < LAG; ++j) wsnap[j] = wlag[j];
                    }
                }
                if (fin_on) {
                    const chunk16* cc = colf[u & 1];
                    CT g = mk<T>(0, 0);
                    if (MODE == MODE_FWD) {
                        double2 gv = ra[u];
                        if (!full_f) gv = csub<double>(gv, ccast<double, T>(cmul<T>(colscalar(cc, XCOL_APREV), ypart)));
                        g = csel<T>(full_f ? act : slot, ccast<T, double>(gv), mk<T>(0, 0));
                    } else if (MODE == MODE_BWD) {
                        g = csel<T>(slot, cmul<T>(colscalar(cc, XCOL_ANEXT), csel<T>(i == 0, ccast<T, double>(ra[u]), ypart)), mk<T>(0, 0));
                    } else if (MODE == MODE_MID) {
                        double2 gv = ra[u];
                        gv = csub<double>(gv, cmul<double>(ccast<double, T>(colscalar(cc, XCOL_APREV)), rb2[u]));
                        gv = csub<double>(gv, cmul<double>(ccast<double, T>(colscalar(cc, XCOL_ANEXT)), rc[u]));
                        g = csel<T>(slot, ccast<T, double>(gv), mk<T>(0, 0));
                    } else {
                        g = csel<T>(act, ccast<T, double>(ra[u]), mk<T>(0, 0));
                    }
                    z = csel<T>(k == 0, g, cfms<T>(cmul<T>(colscalar(cprev, XCOL_E), is2f), w, g));
                }
                prefetch(u, rbk[u], rfk[u], rsp[u], ra[u], rb2[u], rc[u]);
            });
            prefetch_next_group();
        }
    }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------

template <class T, class TF, class TI, class TO, int BV, int MODE>
static bool sweep_bs(int ks, const ProbDev* probs, const ChainDev* chains, int nblocks, const IoDev* io, IoDev iov,
                     C2<T>* sp, const int32_t* act, const SubArg& sa, hipStream_t s) {
    constexpr int Q = RowsOf<BV>::Q, DV = Ring<T, BV>::D;
    dim3 g(nblocks), b(64);
    if (ks == 1) {
        hipLaunchKernelGGL((k_sweep<T, TF, TI, TO, BV, MODE, DV, 1>), g, b, 0, s, probs, chains, io, iov, sp, act, sa);
        return true;
    }
    if constexpr (Q >= 4) {
        if (ks == 2) {
            hipLaunchKernelGGL((k_sweep<T, TF, TI, TO, BV, MODE, DV, 2>), g, b, 0, s, probs, chains, io, iov, sp, act, sa);
            return true;
        }
    }
    if constexpr (Q >= 2) {
        if (ks == Q) {
            hipLaunchKernelGGL((k_sweep<T, TF, TI, TO, BV, MODE, DV, Q>), g, b, 0, s, probs, chains, io, iov, sp, act, sa);
            return true;
        }
    }
    return false;
}

template <class T, class TF, class TI, class TO, int MODE>
static bool sweep_typed(int bs, int ks, const ProbDev* probs, const ChainDev* chains, int nblocks, const IoDev* io,
                        IoDev iov, void* spill, const int32_t* act, const SubArg& sa, hipStream_t s) {
    C2<T>* sp = (C2<T>*)spill;
    switch (bs) {
#define HS_CASE(BV) \
    case BV: return sweep_bs<T, TF, TI, TO, BV, MODE>(ks, probs, chains, nblocks, io, iov, sp, act, sa, s);
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17) HS_CASE(25) HS_CASE(33)
#undef HS_CASE
        default: return false;
    }
}

template <int MODE>
static bool sweep_prec(int bs, int ks, int prec, int in_prec, int out_prec, const ProbDev* probs, const ChainDev* chains,
                       int nb, const IoDev* io, IoDev iov, void* spill, const int32_t* act, const SubArg& sa,
                       hipStream_t s) {
    if (prec == 0) {
        if (in_prec == 0 && out_prec == 0)
            return sweep_typed<double, double, double2, double2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, sa, s);
        return false;
    }
    if (in_prec == 0 && out_prec == 0)
        return sweep_typed<float, float, double2, double2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, sa, s);
    if (in_prec == 0 && out_prec == 1)
        return sweep_typed<float, float, double2, float2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, sa, s);
    if (in_prec == 1 && out_prec == 1)
        return sweep_typed<float, float, float2, float2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, sa, s);
    return false;
}

bool launch_chains(int B, int prec, int in_prec, int out_prec, int phase, int ksplit, const ProbDev* probs,
                   const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill,
                   const int32_t* active, hipStream_t s) {
    if (nchains <= 0) return true;
    SubArg sa{};
    return phase == 0 ? sweep_prec<MODE_FWD>(B, ksplit, prec, in_prec, out_prec, probs, chains, nchains, io, io_val,
                                             spill, active, sa, s)
                      : sweep_prec<MODE_BWD>(B, ksplit, prec, in_prec, out_prec, probs, chains, nchains, io, io_val,
                                             spill, active, sa, s);
}

bool launch_middle(int B, int prec, int in_prec, int out_prec, int ksplit, const ProbDev* probs, const ChainDev* mids,
                   int nmids, const IoDev* io, IoDev io_val, void* spill, const int32_t* active, hipStream_t s) {
    if (nmids <= 0) return true;
    SubArg sa{};
    return sweep_prec<MODE_MID>(2 * B - 1, ksplit, prec, in_prec, out_prec, probs, mids, nmids, io, io_val, spill,
                                active, sa, s);
}

int chain_padded_rows(int B) { return B <= 16 ? 16 : (B <= 32 ? 32 : 64); }
int chain_rhs_per_wave(int B) { return 64 / chain_padded_rows(B); }
int middle_rhs_per_wave(int B) { return 64 / chain_padded_rows(2 * B - 1); }

bool launch_subsolve(int bs, int prec, const ProbDev* prob, const void* fac, const double2* ris2, int rstep, int cdir,
                     int jl, const void* g, void* x, int nrhs, void* spill, hipStream_t s) {
    const int Q = 64 / chain_padded_rows(bs);      // no k-split: one right-hand side per row group
    SubArg sa{fac, (const double2*)g, (double2*)x, ris2, nrhs, rstep, cdir, jl};
    IoDev none{nullptr, nullptr, nullptr};
    const int nb = (nrhs + Q - 1) / Q;
    if (prec == 0) return sweep_typed<double, double, double2, double2, MODE_SUB>(bs, 1, prob, nullptr, nb, nullptr, none, spill, nullptr, sa, s);
    return sweep_typed<float, float, double2, double2, MODE_SUB>(bs, 1, prob, nullptr, nb, nullptr, none, spill, nullptr, sa, s);
}

}  // namespace hs
