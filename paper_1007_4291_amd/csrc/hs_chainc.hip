// a3 / a4 for the moving layers with every strip solve in compressed form.
//
// A moving layer's subproblem (Section 2.2) is only ever used as T~_m: input in its layer row, output
// in its layer row (Algorithm 4: the diagonal applications and both substitutions touch T~_m g with g
// placed in the layer row and read back from it).  Over one strip, T~_m is an n x n map whose
// interaction between distant columns passes through the strip's B-row cross-section, so it is exactly
// represented by per-segment operators of rank B (the structure of the block LU over the strip's
// columns).  For physical segment s (SEG columns, local steps j in the strip's LU order), with the
// strip's block LU recurrences
//   forward:  z_t = e_slot gamma_t + c_t,  c_{t+1} = M_t z_t,         M_t = -E_t diag(1/s2) Lambda_t^{-1}
//   backward: x_t = Lambda_t^{-1} z_t + N_t x_{t+1},  N_t = M_t^T      (Lambda_t^{-1} complex symmetric)
// the segment maps its inputs (gamma on its columns, the carry c_in entering it, the value x_above
// entering its backward pass) to its outputs (layer-row values y, carry out, value leaving backwards):
//   c_out   = Phi c_in + QF gamma
//   x_first = Phi^T x_above + W c_in + QB gamma
//   y       = KS gamma + VS c_in + US x_above
// Running the forward recurrence on the SEG + B unit inputs (gamma = e_j, c_in = e_k) gives
// QF (carries of the gamma inputs at the end), Phi (carries of the c_in inputs), and, accumulating
//   G = sum_t Z_t^T Lambda_t^{-1} Z_t      (Z_t: the z vectors of all unit inputs at step t)
// over the segment, KS = G[gamma, gamma], QB = G[c, gamma], VS = G[gamma, c] = QB^T, W = G[c, c]; the
// x_above response is the transpose of the forward one, US = QF^T (both follow from N_t = M_t^T).
// k_compress forms these blocks in FP64 from the stored factors after every factorisation.
//
// The application of one strip is then, for all right-hand sides of a chain at once:
//   1. per segment:   qf = QF gamma, qb = QB gamma, y = KS gamma
//   2. forward spine: c_in of every segment, c_in(next) = Phi c_in + qf, in the strip's LU order
//   3. per segment:   qb += W c_in, y += VS c_in
//   4. backward spine: x_above(previous) = Phi^T x_above + qb, in reverse LU order
//   5. per segment:   y += US x_above  -> the strip's layer-row output
// the same operator as the sequential block solve (up to rounding), with a sequential depth of two
// spines of n / SEG steps per strip instead of ~2n steps, and no per-column recurrence on the path.
// F and E (full input and output) and the middle layer stay with the segmented / plain chain kernels.
#include <algorithm>

#include "hs_sweep_util.h"

namespace hs {

// Layout (complex elements) of the compressed block of one physical segment of one moving strip.
template <int BS, int SEG> struct CompShape {
    static constexpr int R1 = 2 * BS + SEG;          // rows of G1 = [QF; QB; KS], one column per gamma_j
    static constexpr int R1P = (R1 + 15) & ~15;
    static constexpr int R2 = BS + SEG;              // rows of G2 = [W; VS], one column per c_in entry
    static constexpr int R2P = (R2 + 15) & ~15;
    static constexpr int R3P = (SEG + 15) & ~15;     // rows of G3 = US, one column per x_above entry
    static constexpr int O_G1 = 0;
    static constexpr int O_G2 = O_G1 + SEG * R1P;
    static constexpr int O_G3 = O_G2 + BS * R2P;
    static constexpr int O_PHI = O_G3 + BS * R3P;    // Phi, row-major
    static constexpr int O_CPL = O_PHI + BS * BS;    // [SEG][2]: layer-row couplings to the previous / next layer
    static constexpr int SIZE = (O_CPL + 2 * SEG + 1) & ~1;   // even: every block and section 16-byte aligned
};

template <int BS, int SEG> __host__ __device__ constexpr bool comp_valid() {
    return BS >= 2 && BS <= 16 && 2 * BS + SEG <= 64 && SEG % 16 == 0;
}

// ---------------------------------------------------------------------------------------------
// factor time: the compressed blocks
// ---------------------------------------------------------------------------------------------
constexpr int COMP_THREADS = 256;

template <class TF, int BS, int SEG>
__global__ __launch_bounds__(COMP_THREADS) void k_compress(const ProbDev* __restrict__ probs,
                                                           const CompDev* __restrict__ work) {
    using SH = CompShape<BS, SEG>;
    // Unit inputs, in this order: c_in e_0..e_{B-1} (columns 0..B-1), then gamma_0..gamma_{SEG-1}
    // (columns B..P-1).  gamma_j enters at local step j, so before it its column of z is zero: at
    // step j only the first B + j + 1 columns are nonzero, and every product below is restricted to
    // the 3-column tiles that reach into them (the others would add exact zeros).
    constexpr int P = SEG + BS;
    constexpr int PT = (P + 2) / 3 * 3;               // ... padded to whole triples of columns (zero columns)
    constexpr int TT = PT / 3;
    constexpr int NGT = TT * (TT + 1) / 2;            // 3 x 3 tiles of the upper triangle of the symmetric G
    constexpr int PACK = packed_size(BS), STRIDE = col_stride<TF>(BS);
    constexpr int SLOT = BS - 1;                      // the layer row (local row order)
    static_assert(NGT <= COMP_THREADS && BS * TT <= COMP_THREADS, "one thread per tile");
    // LDS: the z vectors of all unit inputs (FP64, two buffers: this step's and the next step's), y =
    // Lambda^{-1} z, the step's Lambda^{-1} and -E/s2 (two buffers each: the next column's are written
    // while this one's are read), the layer-row couplings; after the steps G (FP32) takes the place of
    // the second z buffer and y
    constexpr int ZB = BS * PT;                       // complex FP64 values per z / y buffer
    constexpr int GB = (P * (P + 1) + 1) / 2;         // G in complex FP64 units
    constexpr int ZYN = 3 * ZB > ZB + GB ? 3 * ZB : ZB + GB;
    __shared__ double2 zyb[ZYN];                      // z[0], z[1], y; then z[0], G
    __shared__ double2 lam2[2][BS][BS];
    __shared__ double2 ne2[2][BS];
    __shared__ float2 cpl[SEG][2];
    auto zsb = [&](int b) { return reinterpret_cast<double2 (*)[PT]>(zyb + b * ZB); };
    double2 (*const ys)[PT] = reinterpret_cast<double2 (*)[PT]>(zyb + 2 * ZB);
    float2 (*const gram)[P + 1] = reinterpret_cast<float2 (*)[P + 1]>(zyb + ZB);

    const CompDev W = work[blockIdx.x];
    const int tid = threadIdx.x;
    const int n = probs[W.prob].n;
    const int tb = (W.cdir > 0) ? W.seg * SEG : n - W.seg * SEG - SEG;   // LU step of local step 0
    const HS_GLOBAL C2<TF>* fac = gptr((const C2<TF>*)W.fac);

    // the steps inside the strip (the others are columns past its edge)
    const int j_lo = tb < 0 ? -tb : 0, j_hi = n - tb < SEG ? n - tb : SEG;
    // z[0]: the c_in unit inputs and gamma_{j_lo}, which enters at the first step; z[1]: zero
    for (int e = tid; e < 2 * ZB; e += COMP_THREADS) {
        const int r = (e % ZB) / PT, p = (e % ZB) - ((e % ZB) / PT) * PT;
        const bool one = e < ZB && (p == r || (r == SLOT && p == BS + j_lo && j_lo < j_hi));
        zyb[e] = make_double2(one ? 1.0 : 0.0, 0.0);
    }
    for (int e = tid; e < 2 * SEG; e += COMP_THREADS) cpl[e >> 1][e & 1] = make_float2(0.f, 0.f);
    // register tiles: the G tile (rows 3 gi .., columns 3 gj ..) and the y tile (row yr, columns 3 yt ..)
    // of this thread, so that every LDS value read feeds three multiply-adds.  Both are numbered so
    // that the tiles in use at a step are those of the lowest thread indices: y tiles by column tile,
    // G tiles by column tile gj, then row tile gi <= gj.
    int gj = 0;
    while ((gj + 1) * (gj + 2) / 2 <= tid) ++gj;
    const int gi = tid - gj * (gj + 1) / 2;
    const int yt = tid / BS, yr = tid - (tid / BS) * BS;
    double2 gacc[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) gacc[i][k] = make_double2(0.0, 0.0);
    // packed index -> (row, column) of this thread's entry of the stored column
    int pr = 0, pk = 0;
    if (tid < PACK) {
        int e = tid;
        while (e >= BS - pr) { e -= BS - pr; ++pr; }
        pk = pr + e;
    }
    // each step's column of the factor is loaded into registers one step ahead, under the previous
    // step's products
    double2 is2 = make_double2(0.0, 0.0);
    if (tid >= PACK && tid < PACK + BS) is2 = gld(gptr(W.ris2 + W.rstep * (tid - PACK)));
    // this thread's entries of a column: the packed inverse (tid < PACK), -E (next BS), the two layer-row
    // couplings (one thread); the others re-read entry 0
    const int fo0 = tid < PACK ? tid : tid < PACK + BS ? PACK + XCOL_E : tid == PACK + BS ? PACK + XCOL_APREV : 0;
    const int fo1 = tid == PACK + BS ? PACK + XCOL_ANEXT : 0;
    C2<TF> pf0 = {}, pf1 = {};
    if (j_lo < j_hi) {
        const HS_GLOBAL C2<TF>* col = fac + (int64_t)(tb + j_lo) * STRIDE;
        pf0 = gld(col + fo0);
        pf1 = gld(col + fo1);
    }
    // this thread's part of loading a column into the buffers of step parity b
    auto put_col = [&](int j, int b) __attribute__((always_inline)) {
        if (tid < PACK) {
            const double2 d = make_double2((double)pf0.x, (double)pf0.y);
            lam2[b][pr][pk] = d;
            lam2[b][pk][pr] = d;
        } else if (tid < PACK + BS) {
            ne2[b][tid - PACK] = cscale<double>(cmul<double>(make_double2((double)pf0.x, (double)pf0.y), is2), -1.0);
        } else if (tid == PACK + BS) {
            cpl[j][0] = make_float2((float)pf0.x, (float)pf0.y);
            cpl[j][1] = make_float2((float)pf1.x, (float)pf1.y);
        }
    };
    __syncthreads();                                  // the initial z and couplings are in place
    if (j_lo < j_hi) {
        put_col(j_lo, 0);
        if (j_lo + 1 < j_hi) {
            const HS_GLOBAL C2<TF>* col = fac + (int64_t)(tb + j_lo + 1) * STRIDE;
            pf0 = gld(col + fo0);
            pf1 = gld(col + fo1);
        }
    }
    __syncthreads();

    // Two block barriers per step: (A) y = Lambda^{-1} z and the next step's z = (-E/s2) y, with the
    // next column's factor data going into the other buffers; (B) G += z^T y.
    for (int j = j_lo; j < j_hi; ++j) {
        const int cur = (j - j_lo) & 1, nx = cur ^ 1;
        const int ta = (BS + j + 1 + 2) / 3;           // column tiles with a nonzero column at this step
        double2 (*const zc)[PT] = zsb(cur);
        double2 (*const zn)[PT] = zsb(nx);
        const bool more = j + 1 < j_hi;
        // (A) a row and three columns of y per thread, and the same entries of the next z; gamma_{j+1}
        // enters the next z in row SLOT, column BS + j + 1
        if (yt < ta) {
            double2 acc[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = make_double2(0.0, 0.0);
#pragma unroll 4
            for (int k = 0; k < BS; ++k) {
                const double2 l = lam2[cur][yr][k];
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = cfma<double>(l, zc[k][3 * yt + c], acc[c]);
            }
            const double2 nr = ne2[cur][yr];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ys[yr][3 * yt + c] = acc[c];
                const bool entry = more && yr == SLOT && 3 * yt + c == BS + j + 1;
                zn[yr][3 * yt + c] = entry ? make_double2(1.0, 0.0) : cmul<double>(nr, acc[c]);
            }
        }
        // gamma_{j+1}'s column past this step's tiles: no thread above writes it
        if (tid == 0 && more && BS + j + 1 >= 3 * ta) zn[SLOT][BS + j + 1] = make_double2(1.0, 0.0);
        if (more) {
            put_col(j + 1, nx);
            if (j + 2 < j_hi) {
                const HS_GLOBAL C2<TF>* col = fac + (int64_t)(tb + j + 2) * STRIDE;
                pf0 = gld(col + fo0);
                pf1 = gld(col + fo1);
            }
        }
        __syncthreads();
        // (B) G += z^T y over the step, a 3 x 3 tile per thread
        if (gj < ta) {
#pragma unroll 2
            for (int r = 0; r < BS; ++r) {
                double2 za[3], yb[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    za[c] = zc[r][3 * gi + c];
                    yb[c] = ys[r][3 * gj + c];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int k = 0; k < 3; ++k) gacc[i][k] = cfma<double>(za[i], yb[k], gacc[i][k]);
            }
        }
        __syncthreads();
    }
    // the final z (after the last step) into buffer 0, so that G can take buffer 1 and y
    if ((j_hi - j_lo) & 1) {
        for (int e = tid; e < ZB; e += COMP_THREADS) zyb[e] = zyb[ZB + e];
        __syncthreads();
    }
    double2 (*const zs)[PT] = zsb(0);
    // G's upper triangle (a <= b) from the tiles, mirrored
    if (tid < NGT) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int a = 3 * gi + i, b = 3 * gj + k;
                if (a < P && b < P && a <= b) {
                    const float2 v = make_float2((float)gacc[i][k].x, (float)gacc[i][k].y);
                    gram[a][b] = v;
                    gram[b][a] = v;
                }
            }
    }
    __syncthreads();
    // the stored blocks; gamma_j is column BS + j, c_in entry k is column k
    HS_GLOBAL float2* out = gptr((float2*)W.out);
    auto zf = [&](int r, int p) -> float2 { return make_float2((float)zs[r][p].x, (float)zs[r][p].y); };
    const float2 zero = make_float2(0.f, 0.f);
    for (int e = tid; e < SH::SIZE; e += COMP_THREADS) {
        float2 v = zero;
        if (e < SH::O_G2) {
            const int j = e / SH::R1P, i = e - j * SH::R1P;
            if (i < BS) v = zf(i, BS + j);                              // QF[i][j]
            else if (i < 2 * BS) v = gram[i - BS][BS + j];              // QB[i-B][j]
            else if (i < SH::R1) v = gram[i - BS][BS + j];              // KS[i-2B][j]: gamma row i - 2B
        } else if (e < SH::O_G3) {
            const int k = (e - SH::O_G2) / SH::R2P, i = (e - SH::O_G2) - k * SH::R2P;
            if (i < SH::R2) v = gram[i][k];                             // W[i][k] (i < B), VS[i-B][k]
        } else if (e < SH::O_PHI) {
            const int k = (e - SH::O_G3) / SH::R3P, jj = (e - SH::O_G3) - k * SH::R3P;
            if (jj < SEG) v = zf(k, BS + jj);                           // US[jj][k] = QF[k][jj]
        } else if (e < SH::O_CPL) {
            const int r = (e - SH::O_PHI) / BS, k = (e - SH::O_PHI) - r * BS;
            v = zf(r, k);                                               // Phi[r][k]
        } else if (e < SH::O_CPL + 2 * SEG) {
            const int q = e - SH::O_CPL;
            v = cpl[q >> 1][q & 1];
        }
        gst(out + e, v);
    }
}

// ---------------------------------------------------------------------------------------------
// application: one workgroup per chain (problem, front, group of RQ right-hand sides), one wave per
// physical segment of the strips
// ---------------------------------------------------------------------------------------------
template <int BS, int SEG, int RQ> struct ChainCShape {
    // LDS (complex64), per segment: gamma / layer row by column, qf, qb, c_in, x_above, the strip's Phi,
    // and a staging area that holds G2, then G3.  Phi and the staging area are filled by asynchronous
    // global-to-LDS copies in chunks of 128 values, so both are padded to whole chunks.
    using SH = CompShape<BS, SEG>;
    static constexpr int GAM = SEG * RQ;
    static constexpr int VEC = BS * RQ;
    static constexpr int PHIP = (BS * BS + 127) & ~127;
    static constexpr int STG = ((BS * SH::R2P > BS * SH::R3P ? BS * SH::R2P : BS * SH::R3P) + 127) & ~127;
    static constexpr int PER_SEG = GAM + 4 * VEC + PHIP + STG;
    static_assert(PHIP > BS * BS, "the spines' spare slot lies in the padding of the Phi area");
};

// Asynchronous copy of LEN complex64 values (LEN even, src 16-byte aligned) from global memory into this
// wave's LDS area dst (room for LEN rounded up to 128): chunk u of lane l moves values 128u + 2l and
// 128u + 2l + 1 (one 16-byte global-to-LDS load per lane and chunk, written at the lane's own 16 bytes of
// the chunk).  Lanes past the end re-read the first pair, into the padding.  The data is in LDS once
// vmcnt has drained (lds_stage_wait, or an exact vmcnt that covers the copy).
// The copies are issued from inline assembly, out of the compiler's sight: it would otherwise wait for
// every copy in flight (vmcnt(0)) before any later LDS read, since it cannot tell which LDS words a copy
// writes -- which would put a global-memory round trip in front of the spines and of phase 5.  Every
// read of staged data here follows an explicit wait; a compiler-placed vmcnt for a register load only
// gets stricter from copies it does not count.  The LDS base goes in M0, which needs one wait state
// before the copy.
template <int LEN>
__device__ __forceinline__ void lds_stage(float2* dst, const HS_GLOBAL float2* src, int lane) {
    constexpr int NCH = (LEN + 127) / 128;
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float2*)dst);
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
        const int e = 128 * u + 2 * lane;
        const HS_GLOBAL float2* const p = src + (e < LEN ? e : 0);
        asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                     :: "v"(p), "s"(d0 + 128u * 8u * u) : "memory", "m0");
    }
}
__device__ __forceinline__ void lds_stage_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Hand-off between the waves of a chain through LDS flags that carry the strip count: a producer
// publishes its LDS data, then the flag (release); a consumer waits for the flag (acquire).  The fences
// cover LDS only: everything handed over lives in LDS (a global-to-LDS copy that is handed over has been
// waited for before the flag), and a fence over global memory as well would wait for every load and copy
// in flight.  The wait is bounded (about 4 M cycles): a hand-off that never comes ends the wait -- wrong
// results, which the parity tests see, rather than a hung device.
// The flag index is made opaque, so that its LDS address is formed at the use rather than hoisted
// out of the strip loop into a register held across it.
__device__ __forceinline__ void flag_set(int* f, int idx, int v) {
    asm volatile("" : "+v"(idx));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __hip_atomic_store(f + idx, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void flag_wait(const int* f, int idx, int v) {
    asm volatile("" : "+v"(idx));
    for (int spin = 0; spin < (1 << 16); ++spin) {
        if (__hip_atomic_load(f + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= v) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Waits for NF flags spaced by stride (one per producing wave) in one bounded loop.
template <int NF>
__device__ __forceinline__ void flag_wait_all(const int* f, int idx, int stride, int v) {
    asm volatile("" : "+v"(idx));
    for (int spin = 0; spin < (1 << 16); ++spin) {
        bool ok = true;
#pragma unroll
        for (int w = 0; w < NF; ++w)
            ok = ok && __hip_atomic_load(f + idx + w * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= v;
        if (ok) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int BS, int SEG, int MODE, class TI, class TO, int RQ>
__global__ __launch_bounds__(1024) void k_chainC(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                                 const IoDev* __restrict__ io, IoDev io_val,
                                                 const int32_t* __restrict__ active) {
    static_assert(MODE == MODE_FWD || MODE == MODE_BWD, "compressed chains serve the front phases");
    static_assert(comp_valid<BS, SEG>(), "one lane per row of the segment blocks");
    using SH = CompShape<BS, SEG>;
    using LS = ChainCShape<BS, SEG, RQ>;
    extern __shared__ __align__(16) float2 lds[];
    const int nwv = blockDim.x >> 6;
    float2* const gam = lds;                           // [nwv][SEG][RQ]
    float2* const qf = gam + nwv * LS::GAM;            // [nwv][BS][RQ]
    float2* const qb = qf + nwv * LS::VEC;
    float2* const cin = qb + nwv * LS::VEC;
    float2* const xab = cin + nwv * LS::VEC;
    float2* const phl = xab + nwv * LS::VEC;            // [nwv][PHIP]: Phi of each segment, row-major
    float2* const stg = phl + nwv * LS::PHIP;           // [nwv][STG]: G2, then G3, of each segment
    constexpr int NSW = RQ / 2;                         // spine waves (the launch has at least as many)
    // ready flags (strip count): qf and qb of each segment (its wave), c_in and x_above of each segment
    // (per spine wave: each writes its own right-hand sides)
    int* const f_qf = (int*)(stg + nwv * LS::STG);
    int* const f_qb = f_qf + nwv;
    int* const f_cin = f_qb + nwv;                      // [NSW][nwv]
    int* const f_xab = f_cin + NSW * nwv;               // [NSW][nwv]
    for (int e = threadIdx.x; e < (2 + 2 * NSW) * nwv; e += blockDim.x) f_qf[e] = 0;
    __syncthreads();

    const ChainDev ch = chains[blockIdx.x];
    if (ch.nq == 0) return;
    if (active && !any_active(active, ch)) return;
    const ProbDev& P = probs[ch.prob];
    const int n = P.n, cmid = P.c;
    const int L = ch.front == 0 ? P.L_lo : P.L_up;
    const int S = (n + SEG - 1) / SEG;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index: uniform
    int lane = threadIdx.x & 63;      // made opaque at every strip (below): per-lane offsets are recomputed
                                      // in the strip loop rather than held in registers across it
    const bool segw = wv < S;                          // this wave has a segment of the strips
    if (!segw && wv >= NSW) return;                    // neither a segment nor a spine for this wave
    const IoDev IO = io ? io[ch.prob] : io_val;
    const int64_t N = (int64_t)n * n;
    const int dirF = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? BS : n + 1 - BS;
    const int sbase = ch.front == 0 ? 0 : P.L_lo;      // compressed strips of the upper front follow the lower ones
    const HS_GLOBAL float2* const cmp = gptr((const float2*)IO.cmp);
    const HS_GLOBAL TI* const fin = gptr((const TI*)IO.in);
    HS_GLOBAL TO* const uout = gptr((TO*)IO.out);
    const int s = wv;
    constexpr int NQH = 64 / SEG;                      // right-hand-side lanes per column in the input step
    float2* const gs = gam + s * LS::GAM;
    float2* const stg_s = stg + s * LS::STG;

    // A spine: v <- Mat_ss v + add_ss over the segments ss in LU order (up) or reverse LU order, storing
    // the value entering each segment in store[ss]; Mat = Phi (mat 0) or Phi^T (mat 1).  The waves of
    // spine rank sr = 0 .. RQ/2 - 1 take two right-hand sides each.  Lane (half, p, r) = (lane >> 5,
    // (lane >> 4) & 1, lane & 15) holds row r of right-hand side q = 2 sr + p and sums Mat[r][kk] v[kk] over its half of the
    // terms, kk = KH half + j (j < KH): v[kk] comes by DPP row broadcast from lane j of a copy of v that is
    // rotated by KH lanes in the upper half, and the two halves are added across lanes l and l ^ 32.  The
    // next segment's matrix row and addends are read from LDS at the top of each step, under its products.
    auto spine = [&](int mat, bool up, const float2* addv, float2* store, const int* f_in, int* f_out, int tgt,
                     int sr) __attribute__((always_inline)) {
        constexpr int KH = (BS + 1) / 2;
        constexpr int NA = 2;                           // independent partial sums
        const int r = lane & 15, half = lane >> 5, q = 2 * sr + ((lane >> 4) & 1);
        const int rr = r < BS ? r : BS - 1, kk0 = KH * half;
        auto seg_at = [&](int k) { return up ? k : S - 1 - k; };
        // Mat[r][kk0 + j] of segment ss at pbase + ss * PHIP + j * pstep.  Past the block (kk0 + j >= BS)
        // this reads finite values of the padded Phi area (every entry of it is written by the strip's
        // copy, or is the spare slot), and they multiply rows of v that are zero.
        const float2* const pbase = phl + (mat == 0 ? rr * BS + kk0 : rr + kk0 * BS);
        const int pstep = mat == 0 ? 1 : BS;
        static_assert((BS - 1) + (2 * ((BS + 1) / 2) - 1) * BS < LS::PHIP, "row reads stay in the Phi area");
        auto load_row = [&](int ss, float2 (&dst)[KH]) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < KH; ++j) dst[j] = pbase[ss * LS::PHIP + j * pstep];
        };
        float2 ad, pr[KH], pr2[KH];
        float z0 = 0.f;
        asm volatile("" : "+v"(z0));                    // a zero made here, not held (or spilled) across the strips
        float2 v = make_float2(z0, z0);
        // a segment's flag publishes its Phi and addends together: wait before reading either
        flag_wait(f_in, seg_at(0), tgt);
        load_row(seg_at(0), pr);
        ad = addv[(seg_at(0) * BS + rr) * RQ + q];
        // lanes that store nothing (upper half, rows past the block) write a spare slot: the padding of
        // segment 0's Phi area
        float2* const spare = phl + BS * BS;
        // the spine is the strip's critical path: its wave issues ahead of the segment waves on its SIMD
        __builtin_amdgcn_s_setprio(2);
        auto step = [&](int k, float2 (&cur)[KH], float2 (&nxt)[KH]) __attribute__((always_inline)) {
            const int ss = seg_at(k), sn = seg_at(k + 1 < S ? k + 1 : k);
            flag_wait(f_in, sn, tgt);                  // the next segment's Phi and addends are published
            load_row(sn, nxt);
            const float2 adn = addv[(sn * BS + rr) * RQ + q];
            __builtin_amdgcn_sched_barrier(0);
            // the upper half's copy of v, rotated so that lane j holds v[KH + j] (row_ror by 16 - KH)
            float2 vr;
            vr.x = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v.x), __float_as_int(v.x),
                                                              0x120 + (16 - KH), 0xC, 0xF, false));
            vr.y = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v.y), __float_as_int(v.y),
                                                              0x120 + (16 - KH), 0xC, 0xF, false));
            float ax[NA], ay[NA];
            static_for<KH>([&](auto KC) __attribute__((always_inline)) {
                constexpr int j = decltype(KC)::value, a = j % NA;
                if constexpr (j < NA) cmul_rowbcast<j>(ax[a], ay[a], cur[j].x, cur[j].y, vr.x, vr.y);
                else cfma_rowbcast<j>(ax[a], ay[a], cur[j].x, cur[j].y, vr.x, vr.y);
            });
            asm volatile("" ::"v"(v.x), "v"(v.y));     // v stays live: its rotated copy takes new registers
            float sx = ax[0], sy = ay[0];
#pragma unroll
            for (int a = 1; a < NA; ++a) {
                if (a < KH) { sx += ax[a]; sy += ay[a]; }
            }
            sx = xor_sum<32>(sx);
            sy = xor_sum<32>(sy);
            v = r < BS ? make_float2(ad.x + sx, ad.y + sy) : make_float2(0.f, 0.f);
            ad = adn;
            // the value entering the next segment, stored now: its register is not rewritten until the
            // end of the next step, so the store never holds up a step
            if (k + 1 < S) {
                *(half == 0 && r < BS ? &store[(sn * BS + r) * RQ + q] : spare) = v;
                if (lane == 0) flag_set(f_out, sn, tgt);
            }
            (void)ss;
        };
        *(half == 0 && r < BS ? &store[(seg_at(0) * BS + r) * RQ + q] : spare) = v;
        if (lane == 0) flag_set(f_out, seg_at(0), tgt);
        for (int k = 0; k < S; k += 2) {       // two steps per pass: the row buffers swap roles, no copies
            step(k, pr, pr2);
            if (k + 1 < S) step(k + 1, pr2, pr);
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // Global data of a strip is requested in three groups, each a phase ahead of its use.  The first: its
    // couplings, input row and the gamma columns G1 (to registers, in the order they are consumed), right
    // after the previous strip's phase 3 (on the spine waves after the backward spine, which needs their
    // registers), then Phi (straight to LDS) once the backward spine has read the previous Phi.  After
    // phase 1 the c_in block G2 (straight to LDS), which arrives during the forward spine; after phase 3
    // the x_above block G3 (to LDS, in G2's place) and, backward, the output row, which arrive during the
    // backward spine.  Every group issues a fixed number of loads (masked lanes read a valid address), so
    // that a wait for "all but the next strip's first group" is an exact vmcnt.
    auto strip_of = [&](int i) { return MODE == MODE_FWD ? i + 1 : L - i; };     // strip index in its front
    auto strip_blk = [&](int i) -> const HS_GLOBAL float2* {
        return cmp + ((int64_t)(sbase + strip_of(i) - 1) * S + s) * SH::SIZE;
    };
    constexpr int NH0 = RQ / NQH;                      // input values per lane
    int icc, iqh, jj5, l3r;                            // input step: this lane's column and right-hand sides;
    bool l3;                                           // phase 3 / 5: rows B .. R1 of G2 (qb, then y), 2B .. R1 of G3
    auto lane_roles = [&]() __attribute__((always_inline)) {
        icc = lane % SEG;
        iqh = lane / SEG;
        l3 = lane >= BS && lane < SH::R1;
        jj5 = lane >= 2 * BS && lane < SH::R1 ? lane - 2 * BS : 0;
        l3r = l3 ? lane - BS : 0;
    };
    lane_roles();
    constexpr int NREQ = 1 + (MODE == MODE_FWD ? NH0 : 0) + (BS * BS + 127) / 128 + SEG;   // loads of a first group
    float2 cpl_v, g1[SEG];
    double2 fin_v[NH0];
    // the first group of strip i (i < L): registers, then Phi
    auto request = [&](int i) __attribute__((always_inline)) {
        const int st = strip_of(i), cd = (st & 1) ? -1 : 1;
        const HS_GLOBAL float2* const blk = strip_blk(i);
        // the block through a buffer resource: wave-uniform base, per-lane 32-bit offsets (no 64-bit
        // address registers)
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(blk, SH::SIZE * (uint32_t)sizeof(float2));
        buf_ld(cpl_v, rs, (uint32_t)(SH::O_CPL + 2 * (cd > 0 ? icc : SEG - 1 - icc) + (MODE == MODE_FWD ? 0 : 1)) * 8u, 0u);
        if constexpr (MODE == MODE_FWD) {
            const int jl = jF + dirF * st, col = s * SEG + icc;
#pragma unroll
            for (int h = 0; h < NH0; ++h) {
                const int q = iqh + NQH * h;
                const bool ok = col < n && q < ch.nq;
                const double2 f = ld2(fin + (ok ? (int64_t)(ch.rhs0 + q) * N + (int64_t)(jl - 1) * n + col : (int64_t)0));
                fin_v[h] = ok ? f : make_double2(0.0, 0.0);
            }
        }
        const uint32_t v1 = (uint32_t)(SH::O_G1 + (lane < SH::R1P ? lane : 0)) * 8u;
#pragma unroll
        for (int j = 0; j < SEG; ++j) buf_ld(g1[j], rs, v1, (uint32_t)(j * SH::R1P) * 8u);
    };
    auto request_phi = [&](int i) __attribute__((always_inline)) {
        lds_stage<BS * BS>(phl + s * LS::PHIP, strip_blk(i) + SH::O_PHI, lane);
    };
    if (segw) { request(0); request_phi(0); }
    for (int i = 0; i < L; ++i) {
        asm volatile("" : "+v"(lane));
        lane_roles();
        const int st = strip_of(i);                            // strip index in its front (1..L)
        const int jl = jF + dirF * st;                         // layer row
        const int cd = (st & 1) ? -1 : 1;                      // column direction of its block LU
        const HS_GLOBAL float2* const blk = strip_blk(i);
        // phase 3 / 5: this lane's row of the y block and its column
        const int cc5 = cd > 0 ? jj5 : SEG - 1 - jj5;
        const int col5 = s * SEG + cc5;
        const bool out5 = lane >= 2 * BS && lane < SH::R1 && col5 < n;
        float2 uold[MODE == MODE_BWD ? RQ : 1];
        if (segw) {
            // ---- 0. the strip's layer-row input on this segment's columns
            {
                const int col = s * SEG + icc;
    #pragma unroll
                for (int h = 0; h < NH0; ++h) {
                    const int q = iqh + NQH * h;
                    float2 g = make_float2(0.f, 0.f);
                    if (col < n && q < ch.nq) {
                        const int64_t rb = (int64_t)(ch.rhs0 + q) * N;
                        if (MODE == MODE_FWD) {
                            const float2 yp = i == 0 ? ccast<float, double>(ld2(uout + rb + (int64_t)(jl - dirF - 1) * n + col))
                                                     : gs[icc * RQ + q];
                            g = csub<float>(make_float2((float)fin_v[h].x, (float)fin_v[h].y), cmul<float>(cpl_v, yp));
                        } else {
                            const float2 yn = i == 0 ? ccast<float, double>(ld2(uout + rb + (int64_t)(cmid - 1) * n + col))
                                                     : gs[icc * RQ + q];
                            g = cmul<float>(cpl_v, yn);
                        }
                    }
                    gs[icc * RQ + q] = g;
                }
            }
            wave_sync();
            // ---- 1. qf, qb and the local part of y from gamma
            {
                float2 acc[RQ];
    #pragma unroll
                for (int q = 0; q < RQ; ++q) acc[q] = make_float2(0.f, 0.f);
                // in groups of 2 columns, so that only one group's gamma values are in flight from LDS
                static_for<SEG / 2>([&](auto GC) __attribute__((always_inline)) {
                    static_for<2>([&](auto UC) __attribute__((always_inline)) {
                        constexpr int j = 2 * decltype(GC)::value + decltype(UC)::value;
                        const int cc = cd > 0 ? j : SEG - 1 - j;
    #pragma unroll
                        for (int q = 0; q < RQ; ++q) acc[q] = cfma<float>(g1[j], gs[cc * RQ + q], acc[q]);
                    });
                    __builtin_amdgcn_sched_barrier(0);
                });
                // Phi is in LDS (the wait drains the first group: G1 has been used, Phi came last); then the
                // c_in block, to arrive during the forward spine
                lds_stage_wait();
                lds_stage<BS * SH::R2P>(stg_s, blk + SH::O_G2, lane);
                wave_sync();          // every lane has read gamma: the layer-row values y take its place
                if (lane < BS) {
    #pragma unroll
                    for (int q = 0; q < RQ; ++q) qf[(s * BS + lane) * RQ + q] = acc[q];
                } else if (lane < 2 * BS) {
    #pragma unroll
                    for (int q = 0; q < RQ; ++q) qb[(s * BS + lane - BS) * RQ + q] = acc[q];
                } else if (lane < SH::R1) {
                    const int jj = lane - 2 * BS, cc = cd > 0 ? jj : SEG - 1 - jj;
    #pragma unroll
                    for (int q = 0; q < RQ; ++q) gs[cc * RQ + q] = acc[q];
                }
            }
            if (lane == 0) flag_set(f_qf, s, i + 1);      // qf, qb and Phi of this segment are in LDS
        }
        // Both spines of the strip run on the waves of the first NSW segments in its LU order (waves without
        // a segment keep their index as spine rank).  Those segments are the last to receive x_above in
        // the previous strip's backward spine and the first to receive c_in here, so their waves are free
        // when this strip's forward spine can begin, and the next strip's spines, which begin at the other
        // end, run on other waves while this strip's backward spine is still going.
        const int sr = segw ? (cd > 0 ? wv : S - 1 - wv) : wv;
        // ---- 2. forward spine: carries entering every segment, in the strip's LU order; it takes each
        // segment's qf as soon as it is published and publishes each c_in
        if (sr < NSW) spine(0, cd > 0, qf, cin, f_qf, f_cin + sr * nwv, i + 1, sr);
        if (segw) {
            // ---- 3. qb += W c_in, y += VS c_in
            // In the backward phase the current values of the output row are requested first: they arrive
            // while this segment waits for its c_in.
            TO uraw[MODE == MODE_BWD ? RQ : 1];
            if constexpr (MODE == MODE_BWD) {
    #pragma unroll
                for (int q = 0; q < RQ; ++q) {
                    const bool ok = out5 && q < ch.nq;
                    uraw[q] = gld(uout + (ok ? (int64_t)(ch.rhs0 + q) * N + (int64_t)(jl - 1) * n + col5 : (int64_t)0));
                }
            }
            flag_wait_all<NSW>(f_cin, s, nwv, i + 1);
            lds_stage_wait();         // G2 is in LDS, and the output row has arrived
            if constexpr (MODE == MODE_BWD) {
    #pragma unroll
                for (int q = 0; q < RQ; ++q) {
                    const bool ok = out5 && q < ch.nq;
                    uold[q] = ok ? make_float2((float)uraw[q].x, (float)uraw[q].y) : make_float2(0.f, 0.f);
                }
            }
            if (l3) {
                float2 acc[RQ];
    #pragma unroll
                for (int q = 0; q < RQ; ++q) acc[q] = make_float2(0.f, 0.f);
                // rolled: the broadcast c_in values are read from LDS step by step, not all at once
    #pragma unroll 2
                for (int k = 0; k < BS; ++k) {
                    const float2 gk = stg_s[k * SH::R2P + l3r];
    #pragma unroll
                    for (int q = 0; q < RQ; ++q) acc[q] = cfma<float>(gk, cin[(s * BS + k) * RQ + q], acc[q]);
                }
                float2* const d = lane < 2 * BS ? &qb[(s * BS + lane - BS) * RQ]
                                                : &gs[(cd > 0 ? lane - 2 * BS : SEG - 1 - (lane - 2 * BS)) * RQ];
    #pragma unroll
                for (int q = 0; q < RQ; ++q) d[q] = cadd<float>(d[q], acc[q]);
            }
            // the x_above block G3, to arrive during the backward spine
            wave_sync();              // every lane of the wave has read G2: G3 takes its place
            if (lane == 0) flag_set(f_qb, s, i + 1);      // qb of this segment is final
            lds_stage<BS * SH::R3P>(stg_s, blk + SH::O_G3, lane);
        }
        // ---- 4. backward spine: values entering every segment from above, reverse LU
        // order, segment by segment as their qb are published
        if (sr < NSW) spine(1, cd < 0, qb, xab, f_qb, f_xab + sr * nwv, i + 1, sr);
        if (segw) {
            // ---- the next strip's first group (the last strip re-requests its own: a fixed count): the
            // registers now -- a segment wave without a spine is here right after its phase 3 --, Phi once
            // the spines have read this segment's Phi
            request(i + 1 < L ? i + 1 : i);
            // x_above of this segment is in LDS, and the spines have read this segment's Phi and qb
            flag_wait_all<NSW>(f_xab, s, nwv, i + 1);
            request_phi(i + 1 < L ? i + 1 : i);
            // ---- 5. y += US x_above; the strip's layer-row output
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(NREQ) : "memory");   // G3 (and the output row) have landed
            if (lane >= 2 * BS && lane < SH::R1) {
                float2 yl[RQ];
    #pragma unroll
                for (int q = 0; q < RQ; ++q) yl[q] = gs[cc5 * RQ + q];
                // rolled: the broadcast x_above values are read from LDS step by step, not all at once
    #pragma unroll 1
                for (int k = 0; k < BS; ++k) {
                    const float2 gk = stg_s[k * SH::R3P + jj5];
    #pragma unroll
                    for (int q = 0; q < RQ; ++q) yl[q] = cfma<float>(gk, xab[(s * BS + k) * RQ + q], yl[q]);
                }
    #pragma unroll
                for (int q = 0; q < RQ; ++q) {
                    float2 y = yl[q];
                    if constexpr (MODE == MODE_BWD) y = csub<float>(uold[q], y);
                    if (col5 < n && q < ch.nq)
                        gst(uout + (int64_t)(ch.rhs0 + q) * N + (int64_t)(jl - 1) * n + col5, cvt_out<TO, float>(y));
                    gs[cc5 * RQ + q] = y;
                }
            }
            wave_sync();
        }
    }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
bool chainc_supported(int B, int seg) {
    if (seg == 32) return B == 4 || B == 5 || B == 7 || B == 9 || B == 13;
    if (seg == 16) return B == 4 || B == 5 || B == 7 || B == 9 || B == 13;
    return false;
}

int64_t comp_block_elems(int B, int seg) {
#define HS_CASE(BV, SV) \
    if (B == BV && seg == SV) return CompShape<BV, SV>::SIZE;
    HS_CASE(4, 16) HS_CASE(5, 16) HS_CASE(7, 16) HS_CASE(9, 16) HS_CASE(13, 16)
    HS_CASE(4, 32) HS_CASE(5, 32) HS_CASE(7, 32) HS_CASE(9, 32) HS_CASE(13, 32)
#undef HS_CASE
    return 0;
}

template <class TF, int SEG>
static bool compress_typed(int B, const ProbDev* probs, const CompDev* work, int nwork, hipStream_t s) {
    switch (B) {
#define HS_CASE(BV) \
    case BV: hipLaunchKernelGGL((k_compress<TF, BV, SEG>), dim3(nwork), dim3(COMP_THREADS), 0, s, probs, work); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13)
#undef HS_CASE
        default: return false;
    }
}

bool launch_compress(int B, int seg, int prec, const ProbDev* probs, const CompDev* work, int nwork, hipStream_t s) {
    if (nwork <= 0) return true;
    if (!chainc_supported(B, seg)) return false;
    if (prec == 0) return seg == 32 ? compress_typed<double, 32>(B, probs, work, nwork, s)
                                    : compress_typed<double, 16>(B, probs, work, nwork, s);
    return seg == 32 ? compress_typed<float, 32>(B, probs, work, nwork, s)
                     : compress_typed<float, 16>(B, probs, work, nwork, s);
}

size_t chainc_lds_bytes(int B, int seg, int rq, int waves) {
    // ChainCShape<B, seg, rq>::PER_SEG per wave, then the ready flags: (2 + 2 rq / 2) ints per wave
    const int r2p = (B + seg + 15) & ~15, r3p = (seg + 15) & ~15;
    const int phip = (B * B + 127) & ~127;
    const int stg = ((B * r2p > B * r3p ? B * r2p : B * r3p) + 127) & ~127;
    const int per = seg * rq + 4 * B * rq + phip + stg;
    return (size_t)per * waves * sizeof(float2) + (size_t)(2 + rq) * waves * sizeof(int);
}

template <int BS, int SEG, int MODE, class TI, class TO, int RQ>
static void chainc_go(const ProbDev* probs, const ChainDev* chains, int nch, const IoDev* io, IoDev iov, int waves,
                      const int32_t* act, hipStream_t s) {
    const size_t lds = chainc_lds_bytes(BS, SEG, RQ, waves);
    hipLaunchKernelGGL((k_chainC<BS, SEG, MODE, TI, TO, RQ>), dim3(nch), dim3(64 * waves), lds, s, probs, chains, io, iov,
                       act);
}

template <int SEG, int MODE, class TI, class TO, int RQ>
static bool chainc_b(int B, const ProbDev* probs, const ChainDev* chains, int nch, const IoDev* io, IoDev iov, int waves,
                     const int32_t* act, hipStream_t s) {
    switch (B) {
#define HS_CASE(BV) \
    case BV: chainc_go<BV, SEG, MODE, TI, TO, RQ>(probs, chains, nch, io, iov, waves, act, s); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13)
#undef HS_CASE
        default: return false;
    }
}

template <int MODE, class TI, class TO>
static bool chainc_r(int B, int seg, int rq, const ProbDev* probs, const ChainDev* chains, int nch, const IoDev* io,
                     IoDev iov, int waves, const int32_t* act, hipStream_t s) {
    if (seg == 32 && rq == 8) return chainc_b<32, MODE, TI, TO, 8>(B, probs, chains, nch, io, iov, waves, act, s);
    if (seg == 32 && rq == 4) return chainc_b<32, MODE, TI, TO, 4>(B, probs, chains, nch, io, iov, waves, act, s);
    if (seg == 16 && rq == 8) return chainc_b<16, MODE, TI, TO, 8>(B, probs, chains, nch, io, iov, waves, act, s);
    if (seg == 16 && rq == 4) return chainc_b<16, MODE, TI, TO, 4>(B, probs, chains, nch, io, iov, waves, act, s);
    return false;
}

bool launch_chains_comp(int B, int seg, int rq, int in_prec, int out_prec, int phase, const ProbDev* probs,
                        const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, int waves,
                        const int32_t* active, hipStream_t s) {
    if (nchains <= 0) return true;
    waves = std::max(waves, rq / 2);                   // the spines take rq / 2 waves
    if (!chainc_supported(B, seg) || waves < 1 || waves > 16) return false;
    if (chainc_lds_bytes(B, seg, rq, waves) > 160 * 1024) return false;
    if (in_prec == 0 && out_prec == 0)
        return phase == 0 ? chainc_r<MODE_FWD, double2, double2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s)
                          : chainc_r<MODE_BWD, double2, double2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s);
    if (in_prec == 0 && out_prec == 1)
        return phase == 0 ? chainc_r<MODE_FWD, double2, float2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s)
                          : chainc_r<MODE_BWD, double2, float2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s);
    if (in_prec == 1 && out_prec == 1)
        return phase == 0 ? chainc_r<MODE_FWD, float2, float2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s)
                          : chainc_r<MODE_BWD, float2, float2>(B, seg, rq, probs, chains, nchains, io, io_val, waves, active, s);
    return false;
}

}  // namespace hs
