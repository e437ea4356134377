// a1 / a5: PML profiles (eq. sigma), coefficient tables, and the FP64 5-point operator (eq. helmd).
#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

// Damping of a layer occupying [0, eta): (C/eta)((t-eta)/eta)^2, zero from eta on (eq. sigma).
__device__ __forceinline__ double sigma_low(double t, double eta, double C) {
    if (t < 0.0 || t >= eta) return 0.0;
    double u = (t - eta) / eta;
    return (C / eta) * u * u;
}

// s = (1 + i sigma/omega)^{-1} and its reciprocal.
__device__ __forceinline__ void stretch(double sigma, double omega, double2& s, double2& is) {
    double a = sigma / omega;
    double d = 1.0 + a * a;
    s = make_double2(1.0 / d, -a / d);
    is = make_double2(1.0, a);
}

// One thread per table entry.  Layout of the table block (see ProfileLayout in hs_kernels.h).
__global__ void k_profiles(ProfileLayout L, double2* tab, double h, double omega, double eta_p,
                           double eta_m, double C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = L.n, B = L.B;
    double sig;
    double2 s, is;
    if (t < n) {                                   // x1 and x2 nodes ih, i = 1..n
        double x = h * (t + 1);
        sig = sigma_low(x, eta_p, C) + sigma_low(1.0 - x, eta_p, C);
        stretch(sig, omega, s, is);
        tab[L.s1n + t] = s; tab[L.is1n + t] = is;
        tab[L.s2n + t] = s; tab[L.is2n + t] = is;
        return;
    }
    t -= n;
    if (t < n + 1) {                               // half points (k + 1/2)h, k = 0..n
        double x = h * (t + 0.5);
        sig = sigma_low(x, eta_p, C) + sigma_low(1.0 - x, eta_p, C);
        stretch(sig, omega, s, is);
        tab[L.s1h + t] = s; tab[L.s2h + t] = s;
        return;
    }
    t -= n + 1;
    if (t < B) {                                   // moving strip rows: distance (r+1)h from its outer edge
        sig = sigma_low(h * (t + 1), eta_m, C);
        stretch(sig, omega, s, is);
        tab[L.mvn + t] = s; tab[L.imvn + t] = is;
        return;
    }
    t -= B;
    if (t < B + 1) {                               // moving strip half rows (q + 1/2)h
        sig = sigma_low(h * (t + 0.5), eta_m, C);
        stretch(sig, omega, s, is);
        tab[L.mvh + t] = s;
        return;
    }
    t -= B + 1;
    if (t < 2 * B - 1) {                           // middle strip rows, damped from both edges
        sig = sigma_low(h * (t + 1), eta_m, C) + sigma_low(h * (2 * B - 1 - t), eta_m, C);
        stretch(sig, omega, s, is);
        tab[L.mdn + t] = s; tab[L.imdn + t] = is;
        return;
    }
    t -= 2 * B - 1;
    if (t < 2 * B) {                               // middle strip half rows
        sig = sigma_low(h * (t + 0.5), eta_m, C) + sigma_low(h * (2 * B - t - 0.5), eta_m, C);
        stretch(sig, omega, s, is);
        tab[L.mdh + t] = s;
    }
}

// 1/c^2 on the grid; flags a non-finite or non-positive velocity.
__global__ void k_inv_c2(const double* __restrict__ c, double* __restrict__ ic2, int64_t N, int* bad) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    double v = c[t];
    if (!(v > 0.0) || !isfinite(v)) { atomicOr(bad, 1); ic2[t] = 0.0; return; }
    ic2[t] = 1.0 / (v * v);
}

void launch_profiles(const ProfileLayout& L, double2* tab, double h, double omega, double eta_p,
                     double eta_m, double C, hipStream_t s) {
    int total = L.n + (L.n + 1) + L.B + (L.B + 1) + (2 * L.B - 1) + 2 * L.B;
    hipLaunchKernelGGL(k_profiles, dim3((total + 255) / 256), dim3(256), 0, s, L, tab, h, omega, eta_p, eta_m, C);
}

void launch_inv_c2(const double* c, double* ic2, int64_t N, int* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_inv_c2, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, c, ic2, N, bad);
}

// ---------------------------------------------------------------------------------------------
// a5: y = A x (alpha = 0) or y = f - A x, FP64 arithmetic, x complex128 or complex64.
// One thread per grid point, coefficients formed once and reused over the right-hand sides.
// Blocks of several problems are concatenated; blk_start[p] is the first block of problem p.
// ---------------------------------------------------------------------------------------------
constexpr int MV_THREADS = 256;

template <class TX>
__global__ __launch_bounds__(MV_THREADS) void k_matvec(const ProbDev* __restrict__ probs, const MvDev* __restrict__ io,
                                                      MvDev io_val, const int32_t* __restrict__ blk_start, int nprob,
                                                      const int32_t* __restrict__ active) {
    const int b = blockIdx.x;
    int lo = 0, hi = nprob - 1;                       // last p with blk_start[p] <= b
    while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (blk_start[mid] <= b) lo = mid; else hi = mid - 1; }
    const int p = blk_start ? lo : 0;
    const int first = blk_start ? blk_start[p] : 0;
    const ProbDev& P = probs[p];
    const MvDev D = io ? io[p] : io_val;
    const int n = P.n;
    const int64_t N = (int64_t)n * n;
    const int64_t t = (int64_t)(b - first) * MV_THREADS + threadIdx.x;
    if (t >= N) return;
    if (active) {                                     // no right-hand side of this problem left
        bool any = false;
        for (int q = 0; q < D.nrhs; ++q) any = any || active[D.sys0 + q] != 0;
        if (!any) return;
    }
    const int j = (int)(t / n) + 1, i = (int)(t % n) + 1;
    const double ih2 = P.ih2;
    const double2 is1 = P.is1n[i - 1], is2 = P.is2n[j - 1];
    const double2 axl = cscale<double>(cmul<double>(P.s1h[i - 1], is2), ih2);
    const double2 axr = cscale<double>(cmul<double>(P.s1h[i], is2), ih2);
    const double2 ayd = cscale<double>(cmul<double>(P.s2h[j - 1], is1), ih2);
    const double2 ayu = cscale<double>(cmul<double>(P.s2h[j], is1), ih2);
    double2 dg = cscale<double>(cmul<double>(cmul<double>(P.omega2, is1), is2), P.ic2[t]);
    dg = csub<double>(dg, cadd<double>(cadd<double>(axl, axr), cadd<double>(ayd, ayu)));
    const TX* __restrict__ x = (const TX*)D.x;
    double2* __restrict__ y = (double2*)D.y;
    const double2* __restrict__ f = (const double2*)D.f;
    for (int q = 0; q < D.nrhs; ++q) {
        if (active && !active[D.sys0 + q]) continue;      // uniform over the block (one problem)
        const TX* xq = x + q * N;
        double2 acc = cmul<double>(dg, ccast<double, decltype(xq->x)>(xq[t]));
        if (i > 1) acc = cfma<double>(axl, ccast<double, decltype(xq->x)>(xq[t - 1]), acc);
        if (i < n) acc = cfma<double>(axr, ccast<double, decltype(xq->x)>(xq[t + 1]), acc);
        if (j > 1) acc = cfma<double>(ayd, ccast<double, decltype(xq->x)>(xq[t - n]), acc);
        if (j < n) acc = cfma<double>(ayu, ccast<double, decltype(xq->x)>(xq[t + n]), acc);
        if (f) acc = csub<double>(f[q * N + t], acc);
        y[q * N + t] = acc;
    }
}

void launch_matvec(const ProbDev* probs, const MvDev* io, MvDev io_val, const int32_t* blk_start, int nprob,
                   int total_blocks, int x_prec, const int32_t* active, hipStream_t s) {
    if (x_prec == 0)
        hipLaunchKernelGGL(k_matvec<double2>, dim3(total_blocks), dim3(MV_THREADS), 0, s, probs, io, io_val, blk_start, nprob,
                           active);
    else
        hipLaunchKernelGGL(k_matvec<float2>, dim3(total_blocks), dim3(MV_THREADS), 0, s, probs, io, io_val, blk_start, nprob,
                           active);
}

int matvec_blocks(int n) { return (int)(((int64_t)n * n + MV_THREADS - 1) / MV_THREADS); }

}  // namespace hs
