// a3 / a4 with every strip solve partitioned into column segments (a SPIKE-style two-level
// recurrence; the paper solves each strip sequentially over its n columns, Algorithm 4).
//
// One strip solve (the forward / backward substitution of the block LU of the strip's quasi-1D
// problem, block-tridiagonal over its columns in LU order t = 0..n-1) is the pair of affine
// recurrences
//   forward:  z_t = g_t + c_t,  w_t = Lambda_t^{-1} z_t,  c_{t+1} = -(E_t s2^{-1}) o w_t,  c_0 = 0
//   backward: x_t = w_t + N_t x_{t+1},  N_t x = -E_t Lambda_t^{-1} (s2^{-1} o x),  x_n = 0
// (c: the carry into the next column; E_t: the column's x1 coupling, s2^{-1}: the strip's row
// factors).  With M_t = -diag(E_t s2^{-1}) Lambda_t^{-1} the carry obeys c_{t+1} = M_t (g_t + c_t),
// and N_t = M_t^T because Lambda_t^{-1} is complex symmetric.
// The n columns are cut into segments of SEG physical columns.  Over a segment the carry obeys
// c_out = Phi c_in + q (Phi = product of the segment's M_t, q = the carry produced from a zero carry
// in), and the backward map is x_top = Phi^T x_above + p.  A strip solve then runs, for every
// segment at once (one 16-lane row group each):
//   F1  forward pass from a zero carry          -> q             (also keeps g_t in registers)
//   F2  the carries at the segment starts, sequentially over segments (one wave per right-hand side)
//   F3  forward pass from the true carry       -> w_t           (registers)
//   B1  backward pass from a zero value above   -> p
//   B2  the values above the segments, sequentially over segments (Phi^T)
//   B3  backward pass from the true value       -> x_t, the strip's outputs
// so its sequential depth is about 4 SEG + 2 n / SEG steps instead of 2 n.  Consecutive strips of a
// front are chained as in the plain sweep: the layer row of strip i feeds the right-hand side of
// strip i + 1 column by column, and segment s of every strip covers the same physical columns, so
// the row group that produces those values (B3) is the one that consumes them (F1 of the next strip).
//
// The propagators Phi of every segment of every strip are products of stored factor data only and
// are formed after each factorisation (k_prop), in the factor precision, one row-major B x B block
// per segment.  F2 reads the blocks, B2 their transposes.  In FP32 the blocks of the strip in hand
// are staged into LDS while the previous strip's last phase runs, so neither spine waits on global
// memory; in FP64 the spine loads them from global memory a few segments ahead.
#include <algorithm>

#include "hs_sweep_util.h"

namespace hs {

namespace {

__device__ __forceinline__ void wg_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // vmcnt 63, expcnt 7, lgkmcnt 0: LDS writes done
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// first LU step of physical segment s (columns s*SEG+1 .. s*SEG+SEG) of a strip with column direction cd
__host__ __device__ __forceinline__ int seg_tbase(int cd, int n, int s) { return cd > 0 ? s * SEG : n - s * SEG - SEG; }

}  // namespace

// ---------------------------------------------------------------------------------------------
// propagators
// ---------------------------------------------------------------------------------------------
// One wave per (strip, group of Q segments); lane (q, r) holds row r of Phi of segment seg0 + q.
// Phi <- M_t Phi over the segment's columns in LU order.
template <class T, class TF, int BS>
__global__ __launch_bounds__(64) void k_prop(const ProbDev* __restrict__ probs, const PropDev* __restrict__ work) {
    using CT = C2<T>;
    using CF = C2<TF>;
    constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q, PACK = packed_size(BS);
    constexpr int STRIDE = col_stride<TF>(BS);
    __shared__ CT phb[Q][BS][BS];
    const PropDev W = work[blockIdx.x];
    const int lane = threadIdx.x, r = lane % RP, q = lane / RP;
    const int n = probs[W.prob].n;
    const int S = (n + SEG - 1) / SEG;
    const int seg = W.seg0 + q;
    const bool rok = r < BS;
    const int rr = rok ? r : 0;
    const HS_GLOBAL CF* fac = gptr((const CF*)W.fac);
    const CT is2 = ccast<T, double>(gld(gptr(W.ris2 + W.rstep * rr)));
    const int tb = seg_tbase(W.cdir, n, seg);
    CT ph[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) ph[c] = mk<T>(c == r ? 1 : 0, 0);
    for (int j = 0; j < SEG; ++j) {
        const int t = tb + j;
        const bool valid = seg < S && t >= 0 && t < n;
        const int tc = t < 0 ? 0 : (t >= n ? n - 1 : t);
        const HS_GLOBAL CF* col = fac + (int64_t)tc * STRIDE;
        if (rok) {
#pragma unroll
            for (int c = 0; c < BS; ++c) phb[q][r][c] = ph[c];
        }
        wave_sync();
        const CT e = ccast<T, TF>(gld(col + PACK + XCOL_E));
        const CT neps = cscale<T>(cmul<T>(e, is2), (T)-1);
        CT l[BS];   // row rr of Lambda_t^{-1}
#pragma unroll
        for (int k = 0; k < BS; ++k) l[k] = ccast<T, TF>(gld(col + (k >= rr ? packed_index(BS, rr, k) : packed_index(BS, k, rr))));
        // row r of M_t Phi, column by column (the previous Phi is read from LDS)
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            CT acc = mk<T>(0, 0);
#pragma unroll
            for (int k = 0; k < BS; ++k) acc = cfma<T>(l[k], phb[q][k][c], acc);
            if (valid && rok) ph[c] = cmul<T>(neps, acc);
        }
        wave_sync();
    }
    if (seg < S && rok) {
        HS_GLOBAL CF* out = gptr((CF*)W.out) + (int64_t)seg * BS * BS + r * BS;   // row r of the block
#pragma unroll
        for (int c = 0; c < BS; ++c) gst(out + c, ccast<TF, T>(ph[c]));
    }
}

// ---------------------------------------------------------------------------------------------
// segmented chains
// ---------------------------------------------------------------------------------------------
template <class T, class TF, int BS> struct SegShape {
    static constexpr int RP = RowsOf<BS>::RP, Q = RowsOf<BS>::Q;
    static constexpr int CB = col_stride<TF>(BS) * (int)sizeof(C2<TF>);   // bytes per stored column
    static constexpr int N16 = CB / 16;
    static constexpr int NCR = (N16 + RP - 1) / RP;                      // column chunks per lane
    // chunks per row group's staged column: 32 bytes of padding shift the row groups of a half wave
    // to other LDS banks (the packed-row reads of neighbouring row groups otherwise collide)
    static constexpr int CSTR = NCR * RP + 2;
    // exchange vectors: LDS only in FP64 (FP32 takes the vector through row broadcasts)
    static constexpr int XZ = sizeof(T) == 8 ? 64 : 0;
    // LDS bytes per wave: staged columns, exchange vectors, 2 spine vectors per segment slot, layer
    // rows.  (Each spine vector holds the per-segment contributions q / p and the values entering the
    // segments c / x in turn: their lifetimes are separated by barriers.)  After the waves' areas, in
    // FP32 only, the strip's segment propagators, shared by every right-hand side of the workgroup
    // (seg_lds_bytes).
    static constexpr int LDS_FIXED = Q * CSTR * 16 + XZ * (int)sizeof(C2<T>) + 2 * Q * RP * (int)sizeof(C2<T>) +
                                     64 * (int)sizeof(C2<T>);
};

// Workgroups of up to 16 waves in FP32 (128 registers per lane) and 8 in FP64.
template <class T> struct SegWaves { static constexpr int MAX = sizeof(T) == 8 ? 8 : 16; };

template <class T, class TF, class TI, class TO, int BS, int MODE>
__global__ __launch_bounds__(64 * SegWaves<T>::MAX) void k_sweepP(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                                 const IoDev* __restrict__ io, IoDev io_val,
                                                 const int32_t* __restrict__ active, C2<T>* __restrict__ wsp,
                                                 int only_front) {
    static_assert(MODE == MODE_FWD || MODE == MODE_BWD, "segmented chains serve the front phases");
    using CT = C2<T>;
    using CF = C2<TF>;
    using SH = SegShape<T, TF, BS>;
    constexpr int RP = SH::RP, Q = SH::Q, NCR = SH::NCR, CB = SH::CB, CSTR = SH::CSTR;
    static_assert(RP == 16 && BS >= 2, "segmented chains take strips of 2 to 16 rows");
    constexpr int PACK = packed_size(BS);
    constexpr int KJ = RP / Q;            // spine: entries of the k-sum per lane
    constexpr int D = 2;                  // column prefetch distance in steps (divides SEG)
    constexpr int PH = BS * BS;           // complex entries per stored segment propagator
    static_assert(SEG % D == 0, "ring slots must repeat per phase");

    extern __shared__ __align__(16) char smem[];
    const int nw = blockDim.x >> 6;
    chunk16* const colb = (chunk16*)smem;                        // [nw][Q][CSTR]
    CT* const xz = (CT*)(colb + nw * Q * CSTR);                  // [nw][XZ]
    CT* const qv = xz + nw * SH::XZ;                             // [nw*Q][RP], by segment slot: q, then p
    CT* const cv = qv + nw * Q * RP;                             // carries c, then values x above
    CT* const pv = qv;
    CT* const xv = cv;
    CT* const ylay = cv + nw * Q * RP;                           // [nw*64]: layer rows by column
    CF* const phl = (CF*)(ylay + nw * 64);                       // [segments][BS*BS] (FP32 only)
    static_assert(SH::LDS_FIXED % 16 == 0, "the propagator area must stay 16-byte aligned");

    const ChainDev ch = chains[blockIdx.x];
    if (ch.nq == 0) return;                                      // padding entry of the table
    if (active && !any_active(active, ch)) return;               // whole workgroup
    const ProbDev& P = probs[ch.prob];
    const int n = P.n, B = P.B, cmid = P.c;
    // only_front: the front strip (F or E) alone, the moving layers being applied by another kernel
    const int L = only_front ? 0 : (ch.front == 0 ? P.L_lo : P.L_up);
    const int m = L;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane % RP, q = lane / RP;
    const int Wr = ch.wrhs;                    // waves per right-hand side
    const int rl = wv / Wr, wr = wv - rl * Wr;
    const bool live = rl < ch.nq;              // wave-uniform
    if (!live) {
        // no right-hand side for this wave: take part in every barrier of the chain, then leave
        for (int b = 0; b < 4 * m + 4; ++b) wg_barrier();
        return;
    }
    const IoDev IO = io ? io[ch.prob] : io_val;
    const int S = (n + SEG - 1) / SEG;
    const int seg = wr * Q + q;
    const bool segok = seg < S;
    const int sl = wv * Q + q;                 // this row group's segment slot
    const int sbase = rl * Wr * Q;             // slot of segment 0 of this right-hand side
    const bool spine = wr == 0;
    const int sub0 = ch.front == 0 ? 0 : P.L_lo + 1;
    const int64_t N = (int64_t)n * n;
    const bool rok = r < BS;
    const int rr = rok ? r : 0;
    const bool slot = rok && r == B - 1;
    const int rhs = ch.rhs0 + rl;
    const HS_GLOBAL TI* __restrict__ fin = gptr((const TI*)IO.in + rhs * N);
    HS_GLOBAL TO* __restrict__ y = gptr((TO*)IO.out + rhs * N);
    const HS_GLOBAL char* const facbase = gptr((const char*)IO.fac);
    const HS_GLOBAL CF* const propbase = gptr((const CF*)IO.prop);
    CT* const ylr = ylay + rl * Wr * 64;       // this right-hand side's layer row, by column - 1
    chunk16* const cb = colb + (wv * Q + q) * CSTR;
    const CF* const cf = (const CF*)cb;
    CT* const xzq = xz + wv * SH::XZ + q * RP;

    const int dirF = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? B : n + 1 - B;
    // backward phase: the row whose updated values feed the first strip's layer row (the middle
    // layer, or the first moving layer when the front strip runs alone)
    const int jfirst = only_front ? jF + dirF : cmid;
    auto strip_t = [&](int i) __attribute__((always_inline)) { return MODE == MODE_FWD ? i : L - i; };
    auto strip_dir = [&](int i) __attribute__((always_inline)) -> int { return (strip_t(i) & 1) ? -1 : 1; };
    auto strip_row = [&](int i) __attribute__((always_inline)) -> int {
        const int jl = jF + dirF * strip_t(i);
        return strip_t(i) == 0 ? jl - dirF * (B - 1 - rr) : jl;
    };
    CT is2_front, is2_other;
    {
        double2 s2, is2, lo, hi;
        strip_profile(P, SUB_PHYS, jF - dirF * (B - 1), dirF, rr, s2, is2, lo, hi);
        is2_front = ccast<T, double>(is2);
        strip_profile(P, SUB_MOVE, 0, 1, rr, s2, is2, lo, hi);
        is2_other = ccast<T, double>(is2);
    }

    int loff[BS];
#pragma unroll
    for (int k = 0; k < BS; ++k) loff[k] = k >= rr ? packed_index(BS, rr, k) : packed_index(BS, k, rr);
    // Row rr of Lambda^{-1} (staged column) times the row group's vector, whose entry r is this
    // lane's z: in FP32 through row broadcasts, in FP64 through the LDS exchange vector.  Every lane
    // of the wave takes part (no divergent branch around it).  Only lanes r < BS are read as entries
    // of the vector, so the z of the padding lanes needs no masking.
    constexpr bool DPP = sizeof(T) == 4;
    auto rowdot = [&](CT z) __attribute__((always_inline)) -> CT {
        if constexpr (DPP) {
            // all reads of the row first, so that they are in flight together (the scheduler would
            // otherwise trade them for register pressure and wait for each in turn)
            CT lv[BS];
#pragma unroll
            for (int k = 0; k < BS; ++k) lv[k] = ccast<T, TF>(cf[loff[k]]);
            __builtin_amdgcn_sched_barrier(0);
            float a0x, a0y, a1x, a1y;
            static_for<BS>([&](auto KC) __attribute__((always_inline)) {
                constexpr int k = decltype(KC)::value;
                if constexpr (k == 0) cmul_rowbcast<k>(a0x, a0y, lv[k].x, lv[k].y, z.x, z.y);
                else if constexpr (k == 1) cmul_rowbcast<k>(a1x, a1y, lv[k].x, lv[k].y, z.x, z.y);
                else if constexpr (k & 1) cfma_rowbcast<k>(a1x, a1y, lv[k].x, lv[k].y, z.x, z.y);
                else cfma_rowbcast<k>(a0x, a0y, lv[k].x, lv[k].y, z.x, z.y);
            });
            return mk<T>(a0x + a1x, a0y + a1y);
        } else {
            xzq[r] = z;
            wave_sync();
            CT acc0 = mk<T>(0, 0), acc1 = mk<T>(0, 0);
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                const CT l = ccast<T, TF>(cf[loff[k]]);
                if (k & 1) acc1 = cfma<T>(l, xzq[k], acc1);
                else acc0 = cfma<T>(l, xzq[k], acc0);
            }
            return cadd<T>(acc0, acc1);
        }
    };

    // Per-strip sources: the strip's stored columns (buffer resource: out-of-range offsets read
    // zeros), this row group's first LU step, column direction, input / output rows.
    struct Src {
        __amdgpu_buffer_rsrc_t col;
        int tb, cd, row, st;
        uint32_t vb;                 // byte offset of this lane's chunk 0 of column tb
        int c0;                      // column - 1 of step 0; step j: c0 + cd * j, clamped to [0, n)
        int ro;                      // (row - 1) * n: the I/O row's element offset
        CT is2;
    };
    auto src_of = [&](int i) __attribute__((always_inline)) -> Src {
        const int ic = i <= m ? i : m;
        Src s;
        s.st = strip_t(ic);
        s.cd = strip_dir(ic);
        s.tb = seg_tbase(s.cd, n, seg);
        s.row = strip_row(ic);
        s.vb = (uint32_t)s.tb * (uint32_t)CB + (uint32_t)(r * 16);
        s.c0 = s.cd > 0 ? s.tb : n - 1 - s.tb;
        s.ro = (s.row - 1) * n;
        s.is2 = s.st == 0 ? is2_front : is2_other;
        s.col = buf_rsrc(facbase + sizeof(CF) * ((int64_t)(sub0 + s.st) * n * col_stride<TF>(BS)), (uint32_t)(n * CB));
        return s;
    };
    // A step's addresses are formed where they are used: the unrolled phases would otherwise keep
    // every step's offsets live from the top of the strip loop (and spill them).  The empty asm makes
    // the per-strip value opaque at that point.
    auto late = [](auto v) __attribute__((always_inline)) {
        asm volatile("" : "+v"(v));
        return v;
    };
    // column - 1 of step j, clamped to the strip (steps off the strip read its edge column)
    auto colm1 = [&](const Src& s, int j) __attribute__((always_inline)) -> int {
        const int c = late(s.c0) + (s.cd > 0 ? j : -j);
        return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
    };
    // right-hand side (input, complex TI) and output (complex TO) of this lane's system, as buffer
    // resources: every access is an element offset from a per-strip row offset
    const __amdgpu_buffer_rsrc_t rin = buf_rsrc(fin, (uint32_t)(N * (int64_t)sizeof(TI)));
    const __amdgpu_buffer_rsrc_t ryo = buf_rsrc(y, (uint32_t)(N * (int64_t)sizeof(TO)));
    auto ioload = [&](auto tag, __amdgpu_buffer_rsrc_t rs, int e) __attribute__((always_inline)) -> double2 {
        using TX = decltype(tag);
        TX v;
        buf_ld(v, rs, (uint32_t)e * (uint32_t)sizeof(TX), 0);
        if constexpr (sizeof(TX) == 16) return v;
        else return make_double2(v.x, v.y);
    };

    // register ring: the column chunks, one input value and one workspace value per step
    chunk16 rk[D][NCR];
    double2 ra[D];
    CT rg[D];
    // Workspace: the forward product w_t of each step (F3 -> B1, B3), laid out
    // [workgroup][step][thread] so that every access is one coalesced 8- or 16-byte word per lane;
    // the register file cannot hold 16 steps of it besides the rest.  (F3 forms the right-hand side
    // g_t again from its inputs, as F1 did, rather than keeping it here: fewer dirty lines in L2.)
    // The last KW products stay in registers (wl, by group of D steps) instead: in FP64 the last D,
    // for B1, whose loads of them would be issued before F3 stores them (B3 loads all 16); in FP32
    // the last 2 D, for B1 and B3, and then they are not stored at all (fewer lines; in FP64 the
    // registers are needed elsewhere).
    constexpr bool WL3 = sizeof(T) == 4;
    constexpr int KW = WL3 ? 2 * D : D;
    static_assert(KW <= SEG, "register-held products within one segment");
    const __amdgpu_buffer_rsrc_t wrs = buf_rsrc(gptr(wsp) + (int64_t)blockIdx.x * SEG * blockDim.x,
                                                (uint32_t)(SEG * blockDim.x * sizeof(CT)));
    // Slots are packed to the rows that exist: row group g = wv * Q + q keeps row r at g * BS + r.  A
    // padding lane (r >= BS) reads its group's first slot (its value is never used) and stores nothing.
    const uint32_t wlane = (uint32_t)(((wv * Q + q) * BS + rr) * sizeof(CT));
    const uint32_t wstep = (uint32_t)(nw * Q * BS * sizeof(CT));
    CT wl[2][D];
    // A column's coupling scalar (E, or the layer-row couplings), taken from the prefetch ring of the
    // lane that loaded it (a DPP row broadcast instead of an LDS read): entry PACK + W of the column
    // lies in chunk (PACK + W) * sizeof(CF) / 16, which lane chunk % RP holds as ring chunk chunk / RP.
    auto ringscalar = [&](auto WC, int u) __attribute__((always_inline)) -> CT {
        constexpr int W = decltype(WC)::value;
        constexpr int BYTE = (PACK + W) * (int)sizeof(CF);
        constexpr int CH = BYTE / 16, LN = CH % RP, C = CH / RP, DW = (BYTE % 16) / 4;
        const chunk16 v = rk[u][C];
        uint32_t d[sizeof(CF) / 4];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(CF) / 4); ++i)
            d[i] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v[DW + i], 0x150 + LN, 0xF, 0xF, false);
        CF out;
        if constexpr (sizeof(CF) == 8) out = make_float2(__uint_as_float(d[0]), __uint_as_float(d[1]));
        else out = make_double2(__hiloint2double((int)d[1], (int)d[0]), __hiloint2double((int)d[3], (int)d[2]));
        return ccast<T, TF>(out);
    };
    // PK: 1 = F1, 3 = F3, 5 = B1, 7 = B3; j: step of the segment in LU order (runtime), u: ring slot.
    // The phases are loops over groups of D steps (only the ring slot is a compile-time index), which
    // keeps the kernel's code within the instruction cache; fully unrolled it was 84 KB.
    auto issue = [&](auto PKC, int j, auto UC, const Src& s, bool first) __attribute__((always_inline)) {
        constexpr int PK = decltype(PKC)::value, u = decltype(UC)::value;
        const uint32_t vo = late(s.vb) + (uint32_t)j * (uint32_t)CB;
#pragma unroll
        for (int c = 0; c < NCR; ++c) rk[u][c] = buf_ld16(s.col, vo + (uint32_t)(c * RP * 16), 0);
        if constexpr (PK == 1 || PK == 3) {
            if (MODE == MODE_FWD) ra[u] = ioload(TI{}, rin, s.ro + colm1(s, j));
            else if (first) ra[u] = ioload(TO{}, ryo, (jfirst - 1) * n + colm1(s, j));
        } else if constexpr (PK == 7) {
            if (MODE == MODE_BWD) ra[u] = ioload(TO{}, ryo, s.ro + colm1(s, j));
        }
        // B1 takes the last D forward products from registers (their loads would precede the stores)
        if constexpr (PK == 5 || PK == 7) {
            if (j < SEG - KW || (PK == 7 && !WL3)) buf_ld(rg[u], wrs, late(wlane), (uint32_t)j * wstep);
        }
    };
    auto stage = [&](int u) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < NCR; ++c) cb[r + c * RP] = rk[u][c];
    };

#pragma unroll
    for (int u = 0; u < D; ++u) { rg[u] = mk<T>(0, 0); wl[0][u] = mk<T>(0, 0); wl[1][u] = mk<T>(0, 0); }
    CT carry = mk<T>(0, 0), xb = mk<T>(0, 0);

    // one forward step: F1 (PK 1) and F3 (PK 3) build g_t from the input and the previous layer row;
    // F3 stores w_t
    // (full: the strip's rows are all outputs (front strip); wout: this lane's row is an output)
    auto fstep = [&](auto PKC, int j, auto UC, const Src& s, bool first, bool full, bool wout)
                     __attribute__((always_inline)) {
        constexpr int PK = decltype(PKC)::value, u = decltype(UC)::value;
        const int t = late(s.tb) + j;
        const bool valid = segok && (uint32_t)t < (uint32_t)n;
        stage(u);
        wave_sync();
        // cross-lane reads first, with every lane active (a DPP source lane outside the exec mask
        // reads as zero)
        const CT sE = ringscalar(std::integral_constant<int, XCOL_E>{}, u);
        CT g;
        {
            const CT sL = ringscalar(std::integral_constant<int, MODE == MODE_FWD ? XCOL_APREV : XCOL_ANEXT>{}, u);
            const int c = colm1(s, j);
            if (MODE == MODE_FWD) {
                CT gv = ccast<T, double>(ra[u]);
                if (!full) gv = csub<T>(gv, cmul<T>(sL, ylr[c]));
                g = wout ? gv : mk<T>(0, 0);
            } else {
                const CT yp = first ? ccast<T, double>(ra[u]) : ylr[c];
                g = slot ? cmul<T>(sL, yp) : mk<T>(0, 0);
            }
            // g is rounded before the carry is added (no multiply-add across the two), so that F1 and
            // F3 give it the same value
            asm volatile("" : "+v"(g.x), "+v"(g.y));
        }
        const CT w = rowdot(cadd<T>(g, carry));
        const CT ne = cscale<T>(cmul<T>(sE, s.is2), (T)-1);
        if constexpr (PK == 3) {
            if ((j < SEG - KW || !WL3) && rok) buf_st(w, wrs, late(wlane), (uint32_t)j * wstep);
            if (j >= SEG - D) wl[1][u] = w;                     // j - (SEG - D) == u
            else if (KW > D && j >= SEG - KW) wl[0][u] = w;     // j - (SEG - 2 D) == u
        }
        carry = csel<T>(valid, cmul<T>(ne, w), carry);
        wave_sync();
    };
    // one backward step: B1 (PK 5) from a zero value above, B3 (PK 7) writes the strip's outputs
    auto bstep = [&](auto PKC, int j, auto UC, const Src& s, bool wout) __attribute__((always_inline)) {
        constexpr int PK = decltype(PKC)::value, u = decltype(UC)::value;
        const int t = late(s.tb) + j;
        const bool valid = segok && (uint32_t)t < (uint32_t)n;
        stage(u);
        wave_sync();
        const CT sE = ringscalar(std::integral_constant<int, XCOL_E>{}, u);
        const CT v = rowdot(cmul<T>(s.is2, xb));
        CT wj = rg[u];
        if (PK == 5 || WL3) {
            if (j >= SEG - D) wj = wl[1][D - 1 - u];                     // j - (SEG - D) == D - 1 - u
            else if (KW > D && j >= SEG - KW) wj = wl[0][D - 1 - u];     // j - (SEG - 2 D) == D - 1 - u
        }
        const CT xn = cfms<T>(sE, v, wj);
        xb = csel<T>(valid, xn, xb);
        if constexpr (PK == 7) {
            const int c = colm1(s, j);
            const CT yval = MODE == MODE_BWD ? csub<T>(ccast<T, double>(ra[u]), xb) : xb;
            if (valid && wout) buf_st(cvt_out<TO, T>(yval), ryo, (uint32_t)(s.ro + c) * (uint32_t)sizeof(TO), 0);
            if (valid && slot) ylr[c] = yval;
        }
        wave_sync();
    };

    // Phases.  Every step refills its ring slot with the step D later in the sequence
    // F3(i) B1(i) B3(i) F1(i+1) F3(i+1) ...; the last group of a phase prefetches the next phase's
    // first group (a backward phase starts at j = SEG-1, a forward one at 0).
    // hook(position) runs after every step (propagator staging).
    constexpr int NG = SEG / D;
    auto phase_f = [&](auto PKC, const Src& s, bool first, auto NPKC, const Src& ns, bool nfirst, auto&& hook)
                       __attribute__((always_inline)) {
        constexpr int NPK = decltype(NPKC)::value;
        const bool full = s.st == 0;
        const bool wout = full ? rok : slot;
        for (int gi = 0; gi < NG; ++gi) {
            static_for<D>([&](auto UC) __attribute__((always_inline)) {
                constexpr int u = decltype(UC)::value;
                const int j = gi * D + u;
                fstep(PKC, j, UC, s, first, full, wout);
                hook(j);
                if (gi + 1 < NG) issue(PKC, j + D, UC, s, first);
                else issue(NPKC, (NPK == 5 || NPK == 7) ? SEG - 1 - u : u, UC, ns, nfirst);
            });
        }
    };
    auto phase_b = [&](auto PKC, const Src& s, auto NPKC, const Src& ns, bool nfirst, auto&& hook)
                       __attribute__((always_inline)) {
        constexpr int NPK = decltype(NPKC)::value;
        const bool wout = s.st == 0 ? rok : slot;
        for (int gi = 0; gi < NG; ++gi) {
            static_for<D>([&](auto UC) __attribute__((always_inline)) {
                constexpr int u = decltype(UC)::value;
                const int k = gi * D + u;                  // position in the phase
                const int j = SEG - 1 - k;
                bstep(PKC, j, UC, s, wout);
                hook(k);
                if (gi + 1 < NG) issue(PKC, j - D, UC, s, false);
                else issue(NPKC, (NPK == 5 || NPK == 7) ? SEG - 1 - u : u, UC, ns, nfirst);
            });
        }
    };
    auto prime = [&](auto PKC, const Src& s, bool first) __attribute__((always_inline)) {
        static_for<D>([&](auto UC) __attribute__((always_inline)) {
            issue(PKC, (int)decltype(UC)::value, UC, s, first);
        });
    };

    // Propagators of strip i: PS complex per strip (16-byte aligned), block si at si * PH.
    const int PS = (S * PH + 1) & ~1;
    auto phi_strip = [&](int i) __attribute__((always_inline)) -> const HS_GLOBAL CF* {
        return propbase + (int64_t)(sub0 + strip_t(i <= m ? i : m)) * PS;
    };
    // FP32: staging of a strip's blocks into LDS, 16-byte chunk c by live thread c mod T, in eight
    // rounds spread over the steps of the phases before the strip's first spine (round jj loads chunk
    // tid + jj*T into a register and stores it to LDS one round later).
    const int nlive = ch.nq * Wr * 64;         // live waves are the first nq * Wr of the workgroup
    const int npc = PS * (int)sizeof(CF) / 16;
    chunk16 phr = {0, 0, 0, 0};
    const HS_GLOBAL chunk16* phsrc = nullptr;
    auto phi_round = [&](int jj) __attribute__((always_inline)) {
        if constexpr (sizeof(T) == 4) {
            if (jj > 0) {
                const int c = (int)threadIdx.x + (jj - 1) * nlive;
                if (c < npc) ((chunk16*)phl)[c] = phr;
            }
            if (jj < 8) {
                const int c = (int)threadIdx.x + jj * nlive;
                phr = phsrc[c < npc ? c : npc - 1];
            }
        }
    };
    auto phi_begin = [&](int i) __attribute__((always_inline)) {
        phsrc = (const HS_GLOBAL chunk16*)phi_strip(i);
    };

    // Spines: one wave per right-hand side; lane (q, r) sums k = jj*Q + q, the row groups are combined
    // with cross-row sums.  F2 takes row rr of each block, B2 column rr.  FP64 loads the blocks from
    // global memory DS segments ahead.
    constexpr int DS = 2;
    auto spine_run = [&](int i, bool fwd) __attribute__((always_inline)) {
        const int cd = strip_dir(i <= m ? i : m);
        const HS_GLOBAL CF* const gph = phi_strip(i);
        CT* const vin = qv;     // segment contributions q (F2) / p (B2)
        CT* const vout = cv;    // values entering the segments: carries c (F2) / x above (B2)
        auto sidx = [&](int k) __attribute__((always_inline)) -> int {
            const int kc = k < S ? k : S - 1;
            return (fwd == (cd > 0)) ? kc : S - 1 - kc;
        };
        CT pr[DS][KJ];
        auto pload = [&](int u, int k) __attribute__((always_inline)) {
            const int base = sidx(k) * PH;
#pragma unroll
            for (int jj = 0; jj < KJ; ++jj) {
                const int kk = jj * Q + q;
                const int kc = kk < BS ? kk : BS - 1;
                const int e = base + (fwd ? rr * BS + kc : kc * BS + rr);
                CT v;
                if constexpr (sizeof(T) == 4) v = ccast<T, TF>(phl[e]);
                else v = ccast<T, TF>(gld(gph + e));
                pr[u][jj] = csel<T>(rok && kk < BS, v, mk<T>(0, 0));
            }
        };
        static_for<DS>([&](auto UC) __attribute__((always_inline)) { pload(decltype(UC)::value, decltype(UC)::value); });
        CT v = mk<T>(0, 0);
        for (int kb = 0; kb < S; kb += DS) {
            static_for<DS>([&](auto UC) __attribute__((always_inline)) {
                constexpr int u = decltype(UC)::value;
                const int k = kb + u;
                if (k < S) {
                    const int si = sidx(k);
                    CT* const vo = vout + (sbase + si) * RP;
                    if (q == 0) vo[r] = v;
                    wave_sync();
                    CT acc = mk<T>(0, 0);
#pragma unroll
                    for (int jj = 0; jj < KJ; ++jj) acc = cfma<T>(pr[u][jj], vo[jj * Q + q], acc);
                    acc.x = xor_sum<16>(acc.x);
                    acc.y = xor_sum<16>(acc.y);
                    acc.x = xor_sum<32>(acc.x);
                    acc.y = xor_sum<32>(acc.y);
                    v = cadd<T>(acc, vin[(sbase + si) * RP + r]);
                    wave_sync();
                    pload(u, k + DS);
                }
            });
        }
    };

    auto no_hook = [](int) __attribute__((always_inline)) {};
    // prologue: F1 of strip 0 (staging strip 0's propagators every second step), its spine
    Src sc = src_of(0), sn = src_of(1);
    phi_begin(0);
    prime(std::integral_constant<int, 1>{}, sc, true);
    phase_f(std::integral_constant<int, 1>{}, sc, true, std::integral_constant<int, 3>{}, sc, true,
            [&](int pos) __attribute__((always_inline)) {
                if ((pos & 1) == 0) phi_round(pos >> 1);
            });
    phi_round(8);
    qv[sl * RP + r] = csel<T>(rok, carry, mk<T>(0, 0));
    wg_barrier();
    if (spine) spine_run(0, true);
    wg_barrier();
    for (int i = 0; i <= m; ++i) {
        carry = cv[sl * RP + r];
        phase_f(std::integral_constant<int, 3>{}, sc, i == 0, std::integral_constant<int, 5>{}, sc, false, no_hook);
        carry = mk<T>(0, 0);
        xb = mk<T>(0, 0);
        phase_b(std::integral_constant<int, 5>{}, sc, std::integral_constant<int, 7>{}, sc, false, no_hook);
        pv[sl * RP + r] = csel<T>(rok, xb, mk<T>(0, 0));
        wg_barrier();
        if (spine) spine_run(i, false);
        wg_barrier();
        // strip i's propagators are no longer read: stage strip i + 1's during B3(i) and F1(i + 1)
        const bool more = i < m;
        if (more) phi_begin(i + 1);
        xb = xv[sl * RP + r];
        phase_b(std::integral_constant<int, 7>{}, sc, std::integral_constant<int, 1>{}, sn, false,
                [&](int pos) __attribute__((always_inline)) {
                    if (more && (pos & 3) == 0) phi_round(pos >> 2);
                });
        if (more) {
            carry = mk<T>(0, 0);
            phase_f(std::integral_constant<int, 1>{}, sn, false, std::integral_constant<int, 3>{}, sn, false,
                    [&](int pos) __attribute__((always_inline)) {
                        if ((pos & 3) == 0) phi_round(4 + (pos >> 2));
                    });
            phi_round(8);
            qv[sl * RP + r] = csel<T>(rok, carry, mk<T>(0, 0));
            wg_barrier();
            if (spine) spine_run(i + 1, true);
            wg_barrier();
        }
        sc = sn;
        sn = src_of(i + 2);
    }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
bool seg_supported(int B) { return B == 4 || B == 5 || B == 7 || B == 9 || B == 13; }

template <class T, class TF> static size_t seg_lds_typed(int B, int waves, int max_n) {
    int fixed = 0;
    switch (B) {
        case 4: fixed = SegShape<T, TF, 4>::LDS_FIXED; break;
        case 5: fixed = SegShape<T, TF, 5>::LDS_FIXED; break;
        case 7: fixed = SegShape<T, TF, 7>::LDS_FIXED; break;
        case 9: fixed = SegShape<T, TF, 9>::LDS_FIXED; break;
        case 13: fixed = SegShape<T, TF, 13>::LDS_FIXED; break;
        default: return 0;
    }
    const int64_t segs = (max_n + SEG - 1) / SEG;
    const int64_t props = sizeof(T) == 4 ? ((segs * B * B + 1) & ~(int64_t)1) * (int64_t)sizeof(C2<TF>) : 0;
    return (size_t)fixed * waves + (size_t)props;
}
size_t seg_lds_bytes(int prec, int B, int waves, int max_n) {
    return prec == 0 ? seg_lds_typed<double, double>(B, waves, max_n) : seg_lds_typed<float, float>(B, waves, max_n);
}
bool seg_fits(int prec, int B, int waves, int max_n) {
    const int maxw = prec == 0 ? SegWaves<double>::MAX : SegWaves<float>::MAX;
    const size_t lds = seg_lds_bytes(prec, B, waves, max_n);
    return seg_supported(B) && waves >= 1 && waves <= maxw && lds > 0 && lds <= 160 * 1024;
}

template <class T, class TF, class TI, class TO, int BV, int MODE>
static bool segp_launch(const ProbDev* probs, const ChainDev* chains, int nb, const IoDev* io, IoDev iov, int waves,
                        const int32_t* act, void* ws, size_t lds, int only_front, hipStream_t s) {
    if (lds > 160 * 1024) return false;
    hipLaunchKernelGGL((k_sweepP<T, TF, TI, TO, BV, MODE>), dim3(nb), dim3(64 * waves), lds, s, probs, chains, io, iov, act,
                       (C2<T>*)ws, only_front);
    return true;
}

template <class T, class TF, class TI, class TO, int MODE>
static bool segp_typed(int bs, const ProbDev* probs, const ChainDev* chains, int nb, const IoDev* io, IoDev iov,
                       int waves, const int32_t* act, void* ws, size_t lds, int of, hipStream_t s) {
    switch (bs) {
#define HS_CASE(BV) \
    case BV: return segp_launch<T, TF, TI, TO, BV, MODE>(probs, chains, nb, io, iov, waves, act, ws, lds, of, s);
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13)
#undef HS_CASE
        default: return false;
    }
}

template <int MODE>
static bool segp_prec(int bs, int prec, int in_prec, int out_prec, const ProbDev* probs, const ChainDev* chains, int nb,
                      const IoDev* io, IoDev iov, int waves, const int32_t* act, void* ws, size_t lds, int of, hipStream_t s) {
    if (prec == 0) {
        if (in_prec == 0 && out_prec == 0)
            return segp_typed<double, double, double2, double2, MODE>(bs, probs, chains, nb, io, iov, waves, act, ws, lds,
                                                                      of, s);
        return false;
    }
    if (in_prec == 0 && out_prec == 0)
        return segp_typed<float, float, double2, double2, MODE>(bs, probs, chains, nb, io, iov, waves, act, ws, lds, of, s);
    if (in_prec == 0 && out_prec == 1)
        return segp_typed<float, float, double2, float2, MODE>(bs, probs, chains, nb, io, iov, waves, act, ws, lds, of, s);
    if (in_prec == 1 && out_prec == 1)
        return segp_typed<float, float, float2, float2, MODE>(bs, probs, chains, nb, io, iov, waves, act, ws, lds, of, s);
    return false;
}

bool launch_chains_seg(int B, int prec, int in_prec, int out_prec, int phase, const ProbDev* probs,
                       const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, int waves, int max_n,
                       const int32_t* active, void* ws, hipStream_t s, int only_front) {
    if (nchains <= 0) return true;
    if (!seg_fits(prec, B, waves, max_n)) return false;
    const size_t lds = seg_lds_bytes(prec, B, waves, max_n);
    return phase == 0 ? segp_prec<MODE_FWD>(B, prec, in_prec, out_prec, probs, chains, nchains, io, io_val, waves, active,
                                            ws, lds, only_front, s)
                      : segp_prec<MODE_BWD>(B, prec, in_prec, out_prec, probs, chains, nchains, io, io_val, waves, active,
                                            ws, lds, only_front, s);
}

int64_t seg_ws_elems(int nchains, int waves) { return (int64_t)nchains * SEG * 64 * waves; }

template <class T, class TF>
static bool prop_typed(int bs, const ProbDev* probs, const PropDev* work, int nwork, hipStream_t s) {
    switch (bs) {
#define HS_CASE(BV) \
    case BV: hipLaunchKernelGGL((k_prop<T, TF, BV>), dim3(nwork), dim3(64), 0, s, probs, work); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13)
#undef HS_CASE
        default: return false;
    }
}

bool launch_prop(int B, int prec, const ProbDev* probs, const PropDev* work, int nwork, hipStream_t s) {
    if (nwork <= 0) return true;
    return prec == 0 ? prop_typed<double, double>(B, probs, work, nwork, s) : prop_typed<float, float>(B, probs, work, nwork, s);
}

}  // namespace hs
