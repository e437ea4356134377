// a3 / a4 with two waves per chain: the backward pass of strip i-1 and the forward pass of strip i
// (Algorithm 4, one front) run on different waves of one workgroup instead of interleaved in one.
//
// The chain's schedule is the one of the single-wave kernel: pair i = (backward pass of strip i-1,
// forward pass of strip i), n + 1 ticks per pair, consecutive strips in opposite column directions so
// that the backward pass of strip i-1 emits its layer row in the column order in which the forward
// pass of strip i consumes it.  Here wave B runs tick k of pair i at step (i, k) and wave F runs the
// same tick one step later, at (i, k + 1); pairs are padded to at least n + 2 steps so that F's last
// slot of a pair is always idle.  Per step:
//   B: x_k = w_{n-1-k} - Lambda^{-1} (e x_{k-1}) (backward step), stores the layer output, and hands
//      it to F through LDS (slot k & 1);
//   F: w = Lambda^{-1} z (forward step), stores it to the workspace, then z = g - e w with g built
//      from the input and B's layer output of the previous step;
//   one LDS barrier (no wait on global memory).
// Forward products go to a global workspace; B reads those of strip i-1 during pair i.  Those of the
// last D steps are also handed over in LDS: every workspace value B prefetches was stored by F at
// least D steps before, so F's own wait for its ring loads of that step (issued after the store)
// completes the store before a barrier that precedes B's load.
#include "hs_sweep_util.h"

namespace hs {

// Workgroup-wide LDS ordering for one step: this wave's LDS writes complete (lgkmcnt(0)), then the
// barrier.  Outstanding global loads and stores are not waited for.
__device__ __forceinline__ void step_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // vmcnt 63, expcnt 7, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T, class TF, class TI, class TO, int BS, int MODE, int D, int KS>
__global__ __launch_bounds__(128) void k_sweep2(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                               const IoDev* __restrict__ io, IoDev io_val, C2<T>* __restrict__ spill_base,
                                               const int32_t* __restrict__ active) {
    static_assert(MODE == MODE_FWD || MODE == MODE_BWD, "two-wave chains serve the front phases");
    static_assert(D % 2 == 0, "slot parities must be compile-time values");
    using CT = C2<T>;
    using CF = C2<TF>;
    constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q;
    using CC = ColChunks<TF, BS>;
    constexpr int STRIDE = CC::STRIDE, N16 = CC::N16, NCH = CC::NCH;
    constexpr int PACK = packed_size(BS);
    __shared__ chunk16 colb[N16];        // B: column of this step
    __shared__ chunk16 colf[2][N16];     // F: columns of this and the previous step
    __shared__ CT xbx[Q][RP];            // B: exchange vector
    __shared__ CT xfx[Q][RP];            // F: exchange vector
    __shared__ CT xlay[2][64];           // B -> F: layer output, by step parity
    __shared__ CT wring[2][D][64];       // F -> B: last D forward products of a strip, by pair parity

    const int role = threadIdx.x >> 6;   // 0: backward pass (B), 1: forward pass (F); wave-uniform
    const int lane = threadIdx.x & 63, r = lane % RP, q = lane / RP;
    const int rq = q / KS, kg = q % KS;
    constexpr int KMAX = (BS + KS - 1) / KS;
    static_assert(BS + KS - 1 <= RP, "the k-split's last round must stay inside the padded rows");
    const ChainDev ch = chains[blockIdx.x];
    if (active && !any_active(active, ch)) return;   // both waves leave before the first barrier
    const ProbDev& P = probs[ch.prob];
    const IoDev IO = io ? io[ch.prob] : io_val;
    const int n = P.n, B = P.B, cmid = P.c;
    const int L = ch.front == 0 ? P.L_lo : P.L_up;
    const int sub0 = ch.front == 0 ? 0 : P.L_lo + 1;
    const int64_t N = (int64_t)n * n;
    const int nq = ch.nq;
    const bool qok = rq < nq;
    const bool rok = r < BS;
    const bool act = qok && rok;
    const bool own = act && kg == 0;
    const bool slot = act && r == B - 1;
    const bool oslot = slot && kg == 0;
    const int rhs = ch.rhs0 + (qok ? rq : 0);
    const int rr = rok ? r : 0;
    const HS_GLOBAL TI* __restrict__ fin = gptr((const TI*)IO.in + rhs * N);
    HS_GLOBAL TO* __restrict__ y = gptr((TO*)IO.out + rhs * N);
    HS_GLOBAL CT* __restrict__ spill = gptr(spill_base + ch.spill_off);
    HS_GLOBAL char* const dummy = (HS_GLOBAL char*)(spill + (int64_t)2 * n * 64) + 16 * lane;
    const HS_GLOBAL char* const facbase = gptr((const char*)IO.fac);

    // the program: strips 0..m in processing order
    const int dirF = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? B : n + 1 - B;
    const int64_t bstride = (int64_t)n * col_stride<TF>(B);
    const int m = L;
    auto strip_t = [&](int i) __attribute__((always_inline)) { return MODE == MODE_FWD ? i : L - i; };
    auto strip_dir = [&](int i) __attribute__((always_inline)) -> int { return (strip_t(i) & 1) ? -1 : 1; };
    auto strip_fac = [&](int i) __attribute__((always_inline)) -> const HS_GLOBAL char* {
        return facbase + sizeof(CF) * ((int64_t)(sub0 + strip_t(i)) * bstride);
    };
    auto strip_full = [&](int i) __attribute__((always_inline)) -> bool { return strip_t(i) == 0; };
    auto strip_row = [&](int i, bool full) __attribute__((always_inline)) -> int {
        const int jl = jF + dirF * strip_t(i);
        return full ? jl - dirF * (B - 1 - rr) : jl;
    };
    CT is2_front, is2_other;
    {
        double2 s2, is2, lo, hi;
        strip_profile(P, SUB_PHYS, jF - dirF * (B - 1), dirF, rr, s2, is2, lo, hi);
        is2_front = ccast<T, double>(is2);
        strip_profile(P, SUB_MOVE, 0, 1, rr, s2, is2, lo, hi);
        is2_other = ccast<T, double>(is2);
    }
    auto strip_is2 = [&](int i) __attribute__((always_inline)) -> CT { return strip_t(i) == 0 ? is2_front : is2_other; };

    // A pair takes n + 1 ticks for B and the same ticks one step later for F: at least n + 2 steps,
    // padded to whole groups of D.
    const int TP = (n + 2 + D - 1) / D * D;
    const int G = TP / D;
    const int64_t colbytes = (int64_t)sizeof(CF) * STRIDE;

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
            // k >= BS only in the last round of a k-split: the exchange entry there is a zero
            // padding row and the factor offset is clamped to a valid entry
            const int k = kg + KS * jj;
            const CT l = ccast<T, TF>(cf[loff[jj]]);
            const CT t = xv[q][KS == 1 ? jj : k];
            if (jj & 1) acc1 = cfma<T>(l, t, acc1);
            else acc0 = cfma<T>(l, t, acc0);
        }
        CT acc = cadd<T>(acc0, acc1);
        if (RP <= 16 && RP * KS >= 32) { acc.x = xor_sum<16>(acc.x); acc.y = xor_sum<16>(acc.y); }
        if (RP <= 32 && RP * KS >= 64) { acc.x = xor_sum<32>(acc.x); acc.y = xor_sum<32>(acc.y); }
        return acc;
    };
    auto colscalar = [&](const chunk16* colv, int which) __attribute__((always_inline)) -> CT {
        return ccast<T, TF>(((const CF*)colv)[PACK + which]);
    };

    // Each role runs its own loop nest (its own prefetch sequence, so the compiler's waits cover
    // exactly the loads of one group earlier); both execute one barrier per step.  Factor columns and
    // the workspace are read and written through buffer resources (per-lane offset in a register,
    // per-step offset scalar).
    const __amdgpu_buffer_rsrc_t srs = buf_rsrc(spill, (uint32_t)(chain_spill_elems(n) * sizeof(CT)));
    const uint32_t lane_cb = (uint32_t)(lane * sizeof(CT));
    const uint32_t ws_bytes = (uint32_t)(64 * sizeof(CT));               // one workspace step
    const uint32_t dummy_off = (uint32_t)(2 * n) * ws_bytes;             // the slot after the workspace
    const uint32_t strip_bytes = (uint32_t)(n * colbytes);
    uint32_t chunk_off[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) chunk_off[c] = (uint32_t)(c * 64 + lane < N16 ? c * 64 + lane : N16 - 1) * 16u;
    const int nmod = (n - 1) % D;

    auto run = [&](auto RC) __attribute__((always_inline)) {
        constexpr int ROLE = decltype(RC)::value;
        // register ring: the column of this wave's strip; B: workspace value and (backward phase)
        // its own output row of the forward phase; F: the input row
        chunk16 rk[D][NCH];
        CT rsp[D];
        double2 ra[D];

        // Prefetch sources of pair pi (B: strip pi-1, F: strip pi), computed once per pair.  Column
        // and workspace reads past a strip's ends are not clamped: their offset, carried in the
        // per-lane (range-checked) buffer offset, falls outside the resource and reads zeros, or
        // hits workspace entries whose values are never used.  Input rows are plain global loads
        // and clamp their column.
        struct Src {
            __amdgpu_buffer_rsrc_t col;
            uint32_t sp;                 // B: workspace byte offset of strip pi-1
            const HS_GLOBAL TI* frow;    // F, forward phase: input row of strip pi
            const HS_GLOBAL TO* yrow;    // B, backward phase: output row of strip pi-1
            int dir;
        };
        auto src_of = [&](int pi) __attribute__((always_inline)) -> Src {
            const int pc = pi <= m + 1 ? pi : m + 1;
            const int ib = pc >= 1 ? pc - 1 : 0, ifw = pc <= m ? pc : m;
            Src S;
            S.dir = strip_dir(pc);
            S.frow = fin;
            S.yrow = y;
            S.sp = 0;
            if constexpr (ROLE == 0) {
                S.col = buf_rsrc(strip_fac(ib), strip_bytes);
                S.sp = (uint32_t)((ib & 1) * n) * ws_bytes;
                if (MODE == MODE_BWD) S.yrow = y + (int64_t)(strip_row(ib, strip_full(ib)) - 1) * n;
            } else {
                S.col = buf_rsrc(strip_fac(ifw), strip_bytes);
                if (MODE == MODE_FWD) S.frow = fin + (int64_t)(strip_row(ifw, strip_full(ifw)) - 1) * n;
            }
            return S;
        };
        // ring slot u for step pk of the pair described by S (B: tick pk; F: tick pk - 1); CL: the
        // step may lie outside the strip (clamp the input-row column)
        auto prefetch = [&](const Src& S, int pk, int u, auto CLC) __attribute__((always_inline)) {
            constexpr bool CL = decltype(CLC)::value;
            if constexpr (ROLE == 0) {
                const uint32_t back = (uint32_t)(n - 1 - pk);
                const uint32_t coff = back * (uint32_t)colbytes;
#pragma unroll
                for (int c = 0; c < NCH; ++c) rk[u][c] = buf_ld16(S.col, chunk_off[c] + coff, 0);
                buf_ld(rsp[u], srs, lane_cb + S.sp + back * ws_bytes, 0);
                if (MODE == MODE_BWD) {
                    const int k2 = CL ? (pk < n - 1 ? pk : n - 1) : pk;
                    const int col = S.dir > 0 ? k2 + 1 : n - k2;
                    ra[u] = ld2(S.yrow + col - 1);
                }
            } else {
                const uint32_t coff = (uint32_t)(pk - 1) * (uint32_t)colbytes;
#pragma unroll
                for (int c = 0; c < NCH; ++c) rk[u][c] = buf_ld16(S.col, chunk_off[c] + coff, 0);
                const int k2 = CL ? max(0, min(pk - 1, n - 1)) : pk - 1;
                const int col = S.dir > 0 ? k2 + 1 : n - k2;
                if (MODE == MODE_FWD) ra[u] = ld2(S.frow + col - 1);
                else ra[u] = ld2(y + (int64_t)(cmid - 1) * n + col - 1);
            }
        };

        Src cur = src_of(0), nxt = src_of(1);
        static_for<D>([&](auto UC) __attribute__((always_inline)) {
            constexpr int u = decltype(UC)::value;
            prefetch(cur, u, u, std::integral_constant<bool, true>{});
        });

        // B: previous layer-row value; F: z and the last forward product
        CT xcur = mk<T>(0, 0), z = mk<T>(0, 0), w = mk<T>(0, 0);
        // Steady groups: all D ticks of the group and of the next one (which it prefetches) inside
        // the strip, not the first group.  There no boundary condition applies: a wave without a
        // strip in this pair (B in the first pair, F in the last) computes unused values, whose
        // workspace and ring writes go to the parity its partner does not read in this pair.
        const int kb_steady = (n - D) / D - 1;

        for (int i = 0; i <= m + 1; ++i) {
            const bool pb = i >= 1, pf = i <= m;
            const int ib = i >= 1 ? i - 1 : 0, ifw = i <= m ? i : m;
            const int cd = strip_dir(i);
            const bool full_b = strip_full(ib);
            const CT is2b = strip_is2(ib);
            HS_GLOBAL TO* const yrow = y + (int64_t)(strip_row(ib, full_b) - 1) * n;
            const bool wy = pb && (full_b ? own : oslot);
            const bool full_f = strip_full(ifw);
            const CT is2f = strip_is2(ifw);
            const uint32_t spw = (uint32_t)((i & 1) * n) * ws_bytes;    // F: workspace of strip i

            // one step: tick k = kb*D + u of this pair (F: tick k-1); ST: steady group (all D ticks
            // inside the strip, not the first group); the ring slot is then refilled for step pk of
            // the pair described by PS
            auto step = [&](auto UC, auto SC, int kb, const Src& PS, int pk) __attribute__((always_inline)) {
                constexpr int u = decltype(UC)::value;
                constexpr bool ST = decltype(SC)::value;
                const int k = kb * D + u;
                if constexpr (ROLE == 0) {
                    // ---- B: tick k of the backward pass of strip i-1 (step s = n-1-k) ----
                    const bool bon = ST ? pb : (pb && k < n);
                    const int col = cd > 0 ? k + 1 : n - k;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int idx = c * 64 + lane < N16 ? c * 64 + lane : N16 - 1;
                        colb[idx] = rk[u][c];
                    }
                    xbx[q][r] = csel<T>(rok, cmul<T>(is2b, xcur), mk<T>(0, 0));   // padding rows read as zeros
                    wave_sync();
                    CT ws = rsp[u];
                    if constexpr (!ST) {
                        // first group: w_{n-1-u} of strip i-1 from the ring of the previous pair
                        const CT wr = wring[(i + 1) & 1][(nmod - u + D) % D][lane];
                        ws = csel<T>(kb == 0, wr, ws);
                    }
                    const CT xb = cfms<T>(colscalar(colb, XCOL_E), rowdot(colb, xbx), ws);
                    const CT x = csel<T>(!ST && k == 0, ws, xb);
                    const CT yval = MODE == MODE_BWD ? csub<T>(ccast<T, double>(ra[u]), x) : x;
                    gst((ST ? wy : (wy && bon)) ? yrow + col - 1 : (HS_GLOBAL TO*)dummy, cvt_out<TO, T>(yval));
                    if (ST || bon) xcur = x;   // steady: unconditional (first pair: values unused)
                    xlay[u & 1][lane] = yval;
                } else {
                    // ---- F: tick kf = k - 1 of the forward pass of strip i ----
                    const int kf = k - 1;
                    const bool fon = ST || (pf && kf >= 1 && kf <= n);
                    const bool fin_on = ST || (pf && kf >= 0 && kf < n);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int idx = c * 64 + lane < N16 ? c * 64 + lane : N16 - 1;
                        colf[(u + 1) & 1][idx] = rk[u][c];
                    }
                    xfx[q][r] = csel<T>(rok, z, mk<T>(0, 0));
                    wave_sync();
                    const chunk16* cc = colf[(u + 1) & 1];     // column kf
                    const chunk16* cprev = colf[u & 1];       // column kf - 1
                    const CT wf = rowdot(cprev, xfx);          // w_{kf-1}
                    buf_st(wf, srs, lane_cb, fon ? spw + (uint32_t)(kf - 1) * ws_bytes : dummy_off);
                    if (fon) {
                        w = wf;
                        wring[i & 1][(u + D - 2) % D][lane] = wf;    // slot (kf - 1) mod D
                    }
                    if (fin_on) {
                        const CT ypart = xlay[(u + 1) & 1][lane];   // B's output of step k-1 = tick kf
                        CT g = mk<T>(0, 0);
                        if (MODE == MODE_FWD) {
                            CT gv = ccast<T, double>(ra[u]);
                            if (!full_f) gv = csub<T>(gv, cmul<T>(colscalar(cc, XCOL_APREV), ypart));
                            g = (full_f ? act : slot) ? gv : mk<T>(0, 0);
                        } else {
                            g = slot ? cmul<T>(colscalar(cc, XCOL_ANEXT), i == 0 ? ccast<T, double>(ra[u]) : ypart)
                                     : mk<T>(0, 0);
                        }
                        const CT zn = cfms<T>(cmul<T>(colscalar(cprev, XCOL_E), is2f), w, g);
                        z = csel<T>(!ST && kf == 0, g, zn);
                    }
                }
                // F's workspace store above is issued before this step's ring loads (the compiler
                // must not hoist them): completing those loads then implies the store completed
                wave_sync();
                prefetch(PS, pk, u, std::integral_constant<bool, !ST>{});
                step_barrier();
            };
            auto group = [&](auto SC, int kb, const Src& PS, int pkb) __attribute__((always_inline)) {
                static_for<D>([&](auto UC) __attribute__((always_inline)) {
                    step(UC, SC, kb, PS, pkb * D + decltype(UC)::value);
                });
            };
            constexpr auto NS = std::integral_constant<bool, false>{};
            constexpr auto SS = std::integral_constant<bool, true>{};
            group(NS, 0, cur, 1);
            int kb = 1;
            for (; kb <= kb_steady && kb < G - 1; ++kb) group(SS, kb, cur, kb + 1);
            for (; kb < G - 1; ++kb) group(NS, kb, cur, kb + 1);
            group(NS, G - 1, nxt, 0);
            cur = nxt;
            nxt = src_of(i + 2);
        }
    };
    if (role == 0) run(std::integral_constant<int, 0>{});
    else run(std::integral_constant<int, 1>{});
}

// prefetch depth of the two-wave chains (each wave holds only its own strip's ring)
template <class T, int BS> struct Ring2 { static constexpr int D = Ring<T, BS>::D; };

template <class T, class TF, class TI, class TO, int BV, int MODE>
static bool sweep2_bs(int ks, const ProbDev* probs, const ChainDev* chains, int nblocks, const IoDev* io, IoDev iov,
                      C2<T>* sp, const int32_t* act, hipStream_t s) {
    constexpr int Q = RowsOf<BV>::Q, DV = Ring2<T, BV>::D;
    dim3 g(nblocks), b(128);
    if (ks == 1) {
        hipLaunchKernelGGL((k_sweep2<T, TF, TI, TO, BV, MODE, DV, 1>), g, b, 0, s, probs, chains, io, iov, sp, act);
        return true;
    }
    if constexpr (Q >= 4) {
        if (ks == 2) {
            hipLaunchKernelGGL((k_sweep2<T, TF, TI, TO, BV, MODE, DV, 2>), g, b, 0, s, probs, chains, io, iov, sp, act);
            return true;
        }
    }
    if constexpr (Q >= 2) {
        if (ks == Q) {
            hipLaunchKernelGGL((k_sweep2<T, TF, TI, TO, BV, MODE, DV, Q>), g, b, 0, s, probs, chains, io, iov, sp, act);
            return true;
        }
    }
    return false;
}

template <class T, class TF, class TI, class TO, int MODE>
static bool sweep2_typed(int bs, int ks, const ProbDev* probs, const ChainDev* chains, int nblocks, const IoDev* io,
                         IoDev iov, void* spill, const int32_t* act, hipStream_t s) {
    C2<T>* sp = (C2<T>*)spill;
    switch (bs) {
#define HS_CASE(BV) \
    case BV: return sweep2_bs<T, TF, TI, TO, BV, MODE>(ks, probs, chains, nblocks, io, iov, sp, act, s);
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17)
#undef HS_CASE
        default: return false;
    }
}

template <int MODE>
static bool sweep2_prec(int bs, int ks, int prec, int in_prec, int out_prec, const ProbDev* probs,
                        const ChainDev* chains, int nb, const IoDev* io, IoDev iov, void* spill, const int32_t* act,
                        hipStream_t s) {
    if (prec == 0) {
        if (in_prec == 0 && out_prec == 0)
            return sweep2_typed<double, double, double2, double2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, s);
        return false;
    }
    if (in_prec == 0 && out_prec == 0)
        return sweep2_typed<float, float, double2, double2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, s);
    if (in_prec == 0 && out_prec == 1)
        return sweep2_typed<float, float, double2, float2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, s);
    if (in_prec == 1 && out_prec == 1)
        return sweep2_typed<float, float, float2, float2, MODE>(bs, ks, probs, chains, nb, io, iov, spill, act, s);
    return false;
}

bool launch_chains2(int B, int prec, int in_prec, int out_prec, int phase, int ksplit, const ProbDev* probs,
                    const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill,
                    const int32_t* active, hipStream_t s) {
    if (nchains <= 0) return true;
    return phase == 0 ? sweep2_prec<MODE_FWD>(B, ksplit, prec, in_prec, out_prec, probs, chains, nchains, io, io_val,
                                              spill, active, s)
                      : sweep2_prec<MODE_BWD>(B, ksplit, prec, in_prec, out_prec, probs, chains, nchains, io, io_val,
                                              spill, active, s);
}

}  // namespace hs
