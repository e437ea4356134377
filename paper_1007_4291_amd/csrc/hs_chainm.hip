// a3 / a4 with the block products Lambda_t^{-1} [B x R] on the matrix cores (factor precision
// HELM_C64_BF16X3): the plain strip recurrences of Algorithm 4 (Section 2.3), one wave per chain of 16
// right-hand sides, every step's block product as MFMA products in bf16x3 form.
//
// bf16x3: an FP32 value x is carried as hi = bf16(x) and lo = bf16(x - hi); a real product a * b is
// formed as lo_a hi_b + hi_a lo_b + hi_a hi_b with FP32 accumulation (Henry, Tang and Heinecke,
// ARITH 2019).  x - (hi + lo) is below 2^-16 |x|, so each product carries a relative error of about
// 2^-16, against 2^-24 for the FP32 products of the HELM_C64 path.
//
// A strip solve (B rows, n columns in the strip's block-LU order t = 0..n-1, Section 2.2) is
//   forward   z_0 = g_0,  w_t = Lambda_t^{-1} z_t,  z_{t+1} = g_{t+1} - E_t is2 o w_t
//   backward  x_{n-1} = w_{n-1},  x_t = w_t - E_t Lambda_t^{-1} (is2 o x_{t+1})
// (E_t: the column coupling of the strip's block tridiagonal form, is2: 1/s2 of each row), with g and
// the output x in the layer row (moving layers) or in every row (F / E).  The chain runs the strips of
// one front in the order of a phase, like the plain chain kernel.
//
// Complex products on real matrix cores, v_mfma_f32_16x16x32_bf16 (A 16 x 32, B 32 x 16, D 16 x 16):
// the K index interleaves real and imaginary parts, k = 2 r + p, so that with Lambda = Lr + i Li and
// z = zr + i zi
//   Wr = sum_k A_r[i][k] Z[k],  A_r[i][2r] = Lr[i][r],  A_r[i][2r+1] = -Li[i][r]
//   Wi = sum_k A_i[i][k] Z[k],  A_i[i][2r] = Li[i][r],  A_i[i][2r+1] =  Lr[i][r]
// with Z[2r] = zr[r], Z[2r+1] = zi[r].  K step s (32 values) covers rows r = 16 s .. 16 s + 15 and M tile m
// rows i = 16 m .. 16 m + 15.  Lane l = 16 g + j holds A rows i = 16 m + j with k = 32 s + 8 g + e, the
// B column j (right-hand side) with the same k, and the D rows 16 m + 4 g + q of column j.  So the
// rows a lane receives in D of tile m are exactly the rows it supplies to the B operand of K step m:
// the recurrences need no exchange between lanes.
//
// Lambda^{-1} is stored by the factorisation as packed FP32 complex; after each factorisation
// k_msplit writes a copy of every F / E / moving strip in split form (per packed entry: dword 0 =
// (re_hi | im_hi << 16), dword 1 = (re_lo | im_lo << 16)), from which the A operands of both products
// follow by a sign flip or a half-word rotation per dword.
#include "hs_sweep_util.h"

namespace hs {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

template <int BS> struct MShape {
    static constexpr int MT = (BS + 15) / 16;     // 16-row tiles of a strip block = 32-wide K steps
    static constexpr int WSV = 2 * MT;            // float4 values of one lane's column in the workspace
};

// hi and lo bf16 of x (round to nearest even), as the low half-words of two dwords
__device__ __forceinline__ void bsplit(float x, unsigned& hi, unsigned& lo) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = (unsigned)__builtin_bit_cast(unsigned short, h);
    lo = (unsigned)__builtin_bit_cast(unsigned short, l);
}

// ---------------------------------------------------------------------------------------------
// factor time: split copy of the packed blocks of the F / E / moving strips
// ---------------------------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(256) void k_msplit(const float2* __restrict__ fac, hs_u2* __restrict__ msp, int64_t ncols) {
    constexpr int PACK = packed_size(BS), STRIDE = col_stride<float>(BS);
    const int64_t total = ncols * STRIDE;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % STRIDE);
        const float2 v = gld(gptr(fac + e));
        hs_u2 o;
        if (k < PACK) {
            unsigned rh, rl, ih, il;
            bsplit(v.x, rh, rl);
            bsplit(v.y, ih, il);
            o.x = rh | (ih << 16);
            o.y = rl | (il << 16);
        } else {
            o.x = __float_as_uint(v.x);                         // coupling scalars, unchanged
            o.y = __float_as_uint(v.y);
        }
        gptr(msp)[e] = o;
    }
}

// ---------------------------------------------------------------------------------------------
// application
// ---------------------------------------------------------------------------------------------
template <int BS, int MODE, class TI, class TO>
__global__ __launch_bounds__(64) void k_chainM(const ProbDev* __restrict__ probs, const ChainDev* __restrict__ chains,
                                               const IoDev* __restrict__ io, IoDev io_val, float4* __restrict__ ws_base,
                                               const int32_t* __restrict__ active) {
    static_assert(MODE == MODE_FWD || MODE == MODE_BWD, "front chains");
    static_assert(BS >= 2 && BS <= 32, "two 16-row tiles at most");
    using MS = MShape<BS>;
    constexpr int MT = MS::MT, PACK = packed_size(BS), STRIDE = col_stride<float>(BS);
    constexpr int SLOT = BS - 1, SMT = SLOT / 16, SG = (SLOT % 16) / 4, SQ = SLOT % 4;   // the layer row's lane slot
    const ChainDev ch = chains[blockIdx.x];
    if (ch.nq == 0) return;
    if (active && !any_active(active, ch)) return;
    const ProbDev& P = probs[ch.prob];
    const IoDev IO = io ? io[ch.prob] : io_val;
    const int n = P.n;
    const int L = ch.front == 0 ? P.L_lo : P.L_up;
    const int sub0 = ch.front == 0 ? 0 : P.L_lo + 1;
    const int64_t N = (int64_t)n * n;
    const int lane = threadIdx.x, j = lane & 15, g = lane >> 4;
    const bool qok = j < ch.nq;
    const int rhs = ch.rhs0 + (qok ? j : 0);
    const HS_GLOBAL TI* const fin = gptr((const TI*)IO.in) + (int64_t)rhs * N;
    HS_GLOBAL TO* const uout = gptr((TO*)IO.out) + (int64_t)rhs * N;
    HS_GLOBAL f32x4_t* const ws = gptr((f32x4_t*)ws_base) + ch.spill_off + lane;     // column t, value c: ws[(t * WSV + c) * 64]
    const int dirF = ch.front == 0 ? 1 : -1;
    const int jF = ch.front == 0 ? BS : n + 1 - BS;
    const int64_t bstride = (int64_t)n * STRIDE;
    const HS_GLOBAL float2* const facbase = gptr((const float2*)IO.fac);
    const HS_GLOBAL hs_u2* const mspbase = gptr((const hs_u2*)IO.msp);

    // packed offsets of this lane's A entries Lambda[16 m + j][16 s + 4 g + q] (-1: outside the block)
    int aoff[MT][MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int s = 0; s < MT; ++s)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * m + j, r = 16 * s + 4 * g + q;
                aoff[m][s][q] = (i < BS && r < BS) ? packed_index(BS, i < r ? i : r, i < r ? r : i) : -1;
            }
    // 1/s2 of this lane's rows 16 m + 4 g + q: front strips (physical profile) and moving layers
    float2 is2f[MT][4], is2m[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * m + 4 * g + q, rr = r < BS ? r : BS - 1;
            double2 s2, is2, lo, hi;
            strip_profile(P, SUB_PHYS, jF - dirF * (BS - 1), dirF, rr, s2, is2, lo, hi);
            is2f[m][q] = r < BS ? ccast<float, double>(is2) : make_float2(0.f, 0.f);
            strip_profile(P, SUB_MOVE, 0, 1, rr, s2, is2, lo, hi);
            is2m[m][q] = r < BS ? ccast<float, double>(is2) : make_float2(0.f, 0.f);
        }

    // Operands of one column, requested one column ahead of their use: this lane's split entries of
    // Lambda_t^{-1}, the column coupling E_t, the layer coupling and layer-row values of the input
    // (forward pass of a layer strip), the stored forward product and old output (backward pass).
    struct Col {
        hs_u2 a[MT][MT][4];
        float2 e, cpl, y;
        double2 fv;
        f32x4_t wsv[MS::WSV];
    };
    // W = Lambda^{-1} Z for this wave's 16 right-hand sides from the column's split entries
    auto product = [&](const Col& C, const float2 (&z)[MT][4], float2 (&w)[MT][4]) __attribute__((always_inline)) {
        u32x4_t bh[MT], bl[MT];
#pragma unroll
        for (int s = 0; s < MT; ++s)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned rh, rl, ih, il;
                bsplit(z[s][q].x, rh, rl);
                bsplit(z[s][q].y, ih, il);
                bh[s][q] = rh | (ih << 16);
                bl[s][q] = rl | (il << 16);
            }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            f32x4_t ar = {0.f, 0.f, 0.f, 0.f}, ai = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < MT; ++s) {
                u32x4_t arh, arl, aih, ail;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const hs_u2 v = C.a[m][s][q];
                    arh[q] = v.x ^ 0x80000000u;                         // (Lr_hi, -Li_hi)
                    arl[q] = v.y ^ 0x80000000u;                         // (Lr_lo, -Li_lo)
                    aih[q] = __builtin_amdgcn_alignbit(v.x, v.x, 16);   // (Li_hi, Lr_hi)
                    ail[q] = __builtin_amdgcn_alignbit(v.y, v.y, 16);   // (Li_lo, Lr_lo)
                }
                const bf16x8_t Bh = __builtin_bit_cast(bf16x8_t, bh[s]), Bl = __builtin_bit_cast(bf16x8_t, bl[s]);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, arl), Bh, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, ail), Bh, ai, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, arh), Bl, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, aih), Bl, ai, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, arh), Bh, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, aih), Bh, ai, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) w[m][q] = make_float2(ar[q], ai[q]);
        }
    };

    for (int i = 0; i <= L; ++i) {
        const int st = MODE == MODE_FWD ? i : L - i;        // strip index in its front (0: F / E)
        const bool full = st == 0;
        const int cd = (st & 1) ? -1 : 1;                    // column direction of the strip's block LU
        const int jl = jF + dirF * st;                       // layer row (F / E: the row next to the layers)
        const HS_GLOBAL float2* const fac = facbase + (int64_t)(sub0 + st) * bstride;
        const HS_GLOBAL hs_u2* const msp = mspbase + (int64_t)(sub0 + st) * bstride;
        float2 is2[MT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) is2[m][q] = full ? is2f[m][q] : is2m[m][q];
        // physical row (1-based) of local row r of a full strip
        auto full_row = [&](int r) { return jl - dirF * (BS - 1 - r); };
        // the layer-row input / output of this lane (slot lanes of live right-hand sides)
        const bool io_slot = qok && g == SG && !(MODE == MODE_FWD && full);
        const int64_t yin_row = MODE == MODE_FWD ? jl - dirF - 1 : jl + dirF - 1;

        // requests of column t (0 <= t < n) for the forward (fw) or backward pass
        auto fetch = [&](int t, bool fw, Col& C) __attribute__((always_inline)) {
            const int col = cd > 0 ? t : n - 1 - t;
            const HS_GLOBAL hs_u2* const cs = msp + (int64_t)t * STRIDE;
            const HS_GLOBAL float2* const cc = fac + (int64_t)t * STRIDE;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int o = aoff[m][s][q];
                        C.a[m][s][q] = cs[o >= 0 ? o : 0];
                    }
            C.e = gld(cc + PACK + XCOL_E);
            if (fw) {
                C.cpl = gld(cc + PACK + (MODE == MODE_FWD ? XCOL_APREV : XCOL_ANEXT));
                C.y = ccast<float, double>(ld2(uout + (io_slot ? yin_row * n + col : (int64_t)0)));
                if (MODE == MODE_FWD) C.fv = ld2(fin + (io_slot ? (int64_t)(jl - 1) * n + col : (int64_t)0));
            } else {
#pragma unroll
                for (int c = 0; c < MS::WSV; ++c) C.wsv[c] = ws[((int64_t)t * MS::WSV + c) * 64];
                if (MODE == MODE_BWD) C.y = ccast<float, double>(ld2(uout + (io_slot ? (int64_t)(jl - 1) * n + col : (int64_t)0)));
            }
        };
        auto zero_outside = [&](Col& C) __attribute__((always_inline)) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int s = 0; s < MT; ++s)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (aoff[m][s][q] < 0) C.a[m][s][q] = hs_u2{0u, 0u};
        };

        // ---- forward pass
        float2 w[MT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) w[m][q] = make_float2(0.f, 0.f);
        float2 eprev = make_float2(0.f, 0.f);                // E of the previous column (none at t = 0)
        auto fstep = [&](int t, Col& C, Col& Nx) __attribute__((always_inline)) {
            if (t + 1 < n) fetch(t + 1, true, Nx);
            zero_outside(C);
            const int col = cd > 0 ? t : n - 1 - t;
            float2 z[MT][4];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) z[m][q] = cmul<float>(cscale<float>(cmul<float>(eprev, is2[m][q]), -1.f), w[m][q]);
            if (qok && MODE == MODE_FWD && full) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 16 * m + 4 * g + q;
                        if (r < BS) z[m][q] = cadd<float>(z[m][q], ccast<float, double>(ld2(fin + (int64_t)(full_row(r) - 1) * n + col)));
                    }
            } else if (io_slot) {
                const float2 gv = MODE == MODE_FWD
                                      ? csub<float>(make_float2((float)C.fv.x, (float)C.fv.y), cmul<float>(C.cpl, C.y))
                                      : cmul<float>(C.cpl, C.y);
                z[SMT][SQ] = cadd<float>(z[SMT][SQ], gv);
            }
            product(C, z, w);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    ws[((int64_t)t * MS::WSV + 2 * m + c) * 64] =
                        f32x4_t{w[m][2 * c].x, w[m][2 * c].y, w[m][2 * c + 1].x, w[m][2 * c + 1].y};
            eprev = C.e;
        };
        {
            Col C0, C1;
            fetch(0, true, C0);
            for (int t = 0; t < n; t += 2) {                 // two columns per pass: the buffers swap roles
                fstep(t, C0, C1);
                if (t + 1 < n) fstep(t + 1, C1, C0);
            }
        }

        // ---- backward pass and the strip's output
        float2 x[MT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) x[m][q] = w[m][q];
        auto output = [&](int t, float2 yold) __attribute__((always_inline)) {
            const int col = cd > 0 ? t : n - 1 - t;
            if (qok && full) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 16 * m + 4 * g + q;
                        if (r < BS) {
                            HS_GLOBAL TO* const dst = uout + (int64_t)(full_row(r) - 1) * n + col;
                            float2 y = x[m][q];
                            if (MODE == MODE_BWD) y = csub<float>(ccast<float, double>(ld2(dst)), y);
                            gst(dst, cvt_out<TO, float>(y));
                        }
                    }
            } else if (io_slot) {
                float2 y = x[SMT][SQ];
                if (MODE == MODE_BWD) y = csub<float>(yold, y);
                gst(uout + (int64_t)(jl - 1) * n + col, cvt_out<TO, float>(y));
            }
        };
        auto bstep = [&](int t, Col& C, Col& Nx) __attribute__((always_inline)) {
            if (t >= 1) fetch(t - 1, false, Nx);
            zero_outside(C);
            float2 v[MT][4], p[MT][4];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) v[m][q] = cmul<float>(is2[m][q], x[m][q]);
            product(C, v, p);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const f32x4_t wv = C.wsv[2 * m + c];
                    x[m][2 * c] = csub<float>(make_float2(wv[0], wv[1]), cmul<float>(C.e, p[m][2 * c]));
                    x[m][2 * c + 1] = csub<float>(make_float2(wv[2], wv[3]), cmul<float>(C.e, p[m][2 * c + 1]));
                }
            output(t, C.y);
        };
        {
            Col C0, C1;
            // column n-1: x = w, its old output value
            float2 ylast = make_float2(0.f, 0.f);
            if (MODE == MODE_BWD && io_slot)
                ylast = ccast<float, double>(ld2(uout + (int64_t)(jl - 1) * n + (cd > 0 ? n - 1 : 0)));
            if (n >= 2) fetch(n - 2, false, C0);
            output(n - 1, ylast);
            for (int t = n - 2; t >= 0; t -= 2) {            // two columns per pass: the buffers swap roles
                bstep(t, C0, C1);
                if (t - 1 >= 0) bstep(t - 1, C1, C0);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
bool chainm_supported(int B) { return B == 4 || B == 5 || B == 7 || B == 9 || B == 13 || B == 17; }

int64_t chainm_ws_f4(int n, int B) { return (int64_t)n * 2 * ((B + 15) / 16) * 64; }

bool launch_msplit(int B, const void* fac, void* msp, int64_t ncols, hipStream_t s) {
    if (ncols <= 0) return true;
    const int blocks = (int)std::min<int64_t>(4096, (ncols * col_stride<float>(B) + 255) / 256);
    switch (B) {
#define HS_CASE(BV) \
    case BV: hipLaunchKernelGGL((k_msplit<BV>), dim3(blocks), dim3(256), 0, s, (const float2*)fac, (hs_u2*)msp, ncols); return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17)
#undef HS_CASE
        default: return false;
    }
}

template <int MODE, class TI, class TO>
static bool chainm_b(int B, const ProbDev* probs, const ChainDev* chains, int nch, const IoDev* io, IoDev iov, void* ws,
                     const int32_t* act, hipStream_t s) {
    switch (B) {
#define HS_CASE(BV)                                                                                                     \
    case BV:                                                                                                            \
        hipLaunchKernelGGL((k_chainM<BV, MODE, TI, TO>), dim3(nch), dim3(64), 0, s, probs, chains, io, iov, (float4*)ws, act); \
        return true;
        HS_CASE(4) HS_CASE(5) HS_CASE(7) HS_CASE(9) HS_CASE(13) HS_CASE(17)
#undef HS_CASE
        default: return false;
    }
}

bool launch_chains_mfma(int B, int in_prec, int out_prec, int phase, const ProbDev* probs, const ChainDev* chains,
                        int nchains, const IoDev* io, IoDev io_val, void* ws, const int32_t* active, hipStream_t s) {
    if (nchains <= 0) return true;
    if (!chainm_supported(B)) return false;
    if (in_prec == 0 && out_prec == 0)
        return phase == 0 ? chainm_b<MODE_FWD, double2, double2>(B, probs, chains, nchains, io, io_val, ws, active, s)
                          : chainm_b<MODE_BWD, double2, double2>(B, probs, chains, nchains, io, io_val, ws, active, s);
    if (in_prec == 0 && out_prec == 1)
        return phase == 0 ? chainm_b<MODE_FWD, double2, float2>(B, probs, chains, nchains, io, io_val, ws, active, s)
                          : chainm_b<MODE_BWD, double2, float2>(B, probs, chains, nchains, io, io_val, ws, active, s);
    if (in_prec == 1 && out_prec == 1)
        return phase == 0 ? chainm_b<MODE_FWD, float2, float2>(B, probs, chains, nchains, io, io_val, ws, active, s)
                          : chainm_b<MODE_BWD, float2, float2>(B, probs, chains, nchains, io, io_val, ws, active, s);
    return false;
}

}  // namespace hs
