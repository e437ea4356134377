// a6: building blocks of right-preconditioned flexible GMRES(k) in FP64, batched over systems.
//
// A system is one right-hand side of one problem.  Long-vector kernels run over a flat list of
// tiles (KR_TILE elements of one system each); per-system scalar work (Givens rotations of the
// Hessenberg column, triangular solve) runs one thread per system.  Reductions go through fixed
// per-tile partial sums followed by an ordered per-system sum, so results are deterministic.
#include "hs_common.h"
#include "hs_kernels.h"

namespace hs {

__device__ __forceinline__ int tile_system(const int32_t* __restrict__ tile_start, int nsys, int b) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (tile_start[mid] <= b) lo = mid; else hi = mid - 1; }
    return lo;
}

__device__ __forceinline__ double2 block_sum(double2 v, double2* red) {
    // 256 threads = 4 waves: reduce within a wave, then across waves through LDS
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off);
        v.y += __shfl_xor(v.y, off);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double2 s = red[0];
    for (int k = 1; k < KR_THREADS / 64; ++k) s = cadd<double>(s, red[k]);
    return s;
}

constexpr int PER_THREAD = KR_TILE / KR_THREADS;

// Basis vectors per pass of the dot and update kernels: their loads are issued together (the last
// group re-reads V_j for the missing ones, from cache, and does not use them).
constexpr int KR_GROUP = 4;

// partial[t * stride + i] = sum_tile conj(V_i) w, i = 0..j
__global__ __launch_bounds__(KR_THREADS) void k_multidot(const SysVec* __restrict__ sv, const int32_t* __restrict__ tile_start,
                                                         int nsys, int j, double2* __restrict__ partial, int stride,
                                                         const int32_t* __restrict__ active) {
    __shared__ double2 red[KR_GROUP][KR_THREADS / 64];
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    if (active && !active[s]) return;
    const SysVec V = sv[s];
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
    double2 wv[PER_THREAD];
    int64_t ix[PER_THREAD];
    bool ok[PER_THREAD];
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        ok[e] = idx < V.len;
        ix[e] = ok[e] ? idx : V.len - 1;
        wv[e] = ok[e] ? gld(gptr(V.w) + idx) : make_double2(0.0, 0.0);
    }
    for (int i0 = 0; i0 <= j; i0 += KR_GROUP) {
        double2 a[KR_GROUP][PER_THREAD];
#pragma unroll
        for (int g = 0; g < KR_GROUP; ++g) {
            const HS_GLOBAL double2* vi = gptr(V.v) + (int64_t)min(i0 + g, j) * V.vstride;
#pragma unroll
            for (int e = 0; e < PER_THREAD; ++e) a[g][e] = gld(vi + ix[e]);
        }
        double2 acc[KR_GROUP];
#pragma unroll
        for (int g = 0; g < KR_GROUP; ++g) {
            acc[g] = make_double2(0.0, 0.0);
#pragma unroll
            for (int e = 0; e < PER_THREAD; ++e) {
                if (ok[e]) {
                    acc[g].x = fma(a[g][e].x, wv[e].x, fma(a[g][e].y, wv[e].y, acc[g].x));
                    acc[g].y = fma(a[g][e].x, wv[e].y, fma(-a[g][e].y, wv[e].x, acc[g].y));
                }
            }
            // wave sums, as in block_sum
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                acc[g].x += __shfl_xor(acc[g].x, off);
                acc[g].y += __shfl_xor(acc[g].y, off);
            }
        }
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int g = 0; g < KR_GROUP; ++g) red[g][w] = acc[g];
        }
        __syncthreads();
        if (threadIdx.x < KR_GROUP && i0 + (int)threadIdx.x <= j) {
            const int g = threadIdx.x;
            double2 t = red[g][0];
            for (int k = 1; k < KR_THREADS / 64; ++k) t = cadd<double>(t, red[g][k]);
            partial[(int64_t)b * stride + i0 + g] = t;
        }
    }
}

// h[s * hstride + i] (+)= sum over tiles of system s of partial[t * stride + i]
__global__ void k_reduce_partials(const int32_t* __restrict__ tile_start, const double2* __restrict__ partial, int stride,
                                  int cnt, double2* __restrict__ h, int hstride, int accumulate,
                                  const int32_t* __restrict__ active) {
    const int s = blockIdx.x;
    if (active && !active[s]) return;
    const int t0 = tile_start[s], t1 = tile_start[s + 1];
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int t = t0; t < t1; ++t) acc = cadd<double>(acc, partial[(int64_t)t * stride + i]);
        double2* dst = h + (int64_t)s * hstride + i;
        *dst = accumulate ? cadd<double>(*dst, acc) : acc;
    }
}

// w -= sum_{i<=j} h_i V_i, subtracted in increasing i for every element; with npart, also the tile's
// partial sum of |w|^2 of the result into npart[tile] (as k_norm_partials: same elements, order, tree)
__global__ __launch_bounds__(KR_THREADS) void k_multiaxpy(const SysVec* __restrict__ sv, const int32_t* __restrict__ tile_start,
                                                          int nsys, int j, const double2* __restrict__ h, int hstride,
                                                          const int32_t* __restrict__ active, double2* __restrict__ npart) {
    __shared__ double2 red[KR_THREADS / 64];
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    if (active && !active[s]) return;
    const SysVec V = sv[s];
    const double2* hs_ = h + (int64_t)s * hstride;
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
    double2 acc[PER_THREAD];
    int64_t ix[PER_THREAD];
    bool ok[PER_THREAD];
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        ok[e] = idx < V.len;
        ix[e] = ok[e] ? idx : V.len - 1;
        acc[e] = gld(gptr(V.w) + ix[e]);
    }
    for (int i0 = 0; i0 <= j; i0 += KR_GROUP) {
        double2 a[KR_GROUP][PER_THREAD];
#pragma unroll
        for (int g = 0; g < KR_GROUP; ++g) {
            const HS_GLOBAL double2* vi = gptr(V.v) + (int64_t)min(i0 + g, j) * V.vstride;
#pragma unroll
            for (int e = 0; e < PER_THREAD; ++e) a[g][e] = gld(vi + ix[e]);
        }
#pragma unroll
        for (int g = 0; g < KR_GROUP; ++g) {
            if (i0 + g > j) break;
            const double2 hg = hs_[i0 + g];
#pragma unroll
            for (int e = 0; e < PER_THREAD; ++e) acc[e] = cfms<double>(hg, a[g][e], acc[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e)
        if (ok[e]) gst(gptr(V.w) + ix[e], acc[e]);
    if (npart) {
        double nacc = 0.0;
#pragma unroll
        for (int e = 0; e < PER_THREAD; ++e)
            if (ok[e]) nacc = fma(acc[e].x, acc[e].x, fma(acc[e].y, acc[e].y, nacc));
        const double2 tot = block_sum(make_double2(nacc, 0.0), red);
        if (threadIdx.x == 0) npart[b] = tot;
    }
}

// The first update of a Gram-Schmidt pair fused with the second pass's dot products, for up to
// KR_FUSE basis vectors: per element, the basis values stay in registers between the update
// w -= sum_{i<=j} h_i V_i (subtracted in increasing i, as k_multiaxpy) and the products
// partial[t * stride + i] = sum_tile conj(V_i) w (summed over the elements in order and reduced by
// the same tree as k_multidot), so the pass reads V once instead of twice and gives the same values.
__global__ __launch_bounds__(KR_THREADS) void k_multiaxpy_dot(const SysVec* __restrict__ sv,
                                                              const int32_t* __restrict__ tile_start, int nsys, int j,
                                                              const double2* __restrict__ h, int hstride,
                                                              double2* __restrict__ partial, int stride,
                                                              const int32_t* __restrict__ active) {
    __shared__ double2 red[KR_GROUP][KR_THREADS / 64];
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    if (active && !active[s]) return;
    const SysVec V = sv[s];
    const double2* hs_ = h + (int64_t)s * hstride;
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
    double2 d[KR_FUSE];
#pragma unroll
    for (int i = 0; i < KR_FUSE; ++i) d[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        const bool ok = idx < V.len;
        const int64_t ix = ok ? idx : V.len - 1;
        double2 v[KR_FUSE];
#pragma unroll
        for (int i = 0; i < KR_FUSE; ++i)
            if (i <= j) v[i] = gld(gptr(V.v) + (int64_t)i * V.vstride + ix);
        double2 w = gld(gptr(V.w) + ix);
#pragma unroll
        for (int i = 0; i < KR_FUSE; ++i)
            if (i <= j) w = cfms<double>(hs_[i], v[i], w);
        if (ok) {
            gst(gptr(V.w) + ix, w);
#pragma unroll
            for (int i = 0; i < KR_FUSE; ++i) {
                if (i <= j) {
                    d[i].x = fma(v[i].x, w.x, fma(v[i].y, w.y, d[i].x));
                    d[i].y = fma(v[i].x, w.y, fma(-v[i].y, w.x, d[i].y));
                }
            }
        }
    }
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int i0 = 0; i0 < KR_FUSE; i0 += KR_GROUP) {
        if (i0 > j) break;
#pragma unroll
        for (int g = 0; g < KR_GROUP; ++g) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                d[i0 + g].x += __shfl_xor(d[i0 + g].x, off);
                d[i0 + g].y += __shfl_xor(d[i0 + g].y, off);
            }
        }
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int g = 0; g < KR_GROUP; ++g) red[g][wv] = d[i0 + g];
        }
        __syncthreads();
        if (threadIdx.x < KR_GROUP && i0 + (int)threadIdx.x <= j) {
            const int g = threadIdx.x;
            double2 t = red[g][0];
            for (int k = 1; k < KR_THREADS / 64; ++k) t = cadd<double>(t, red[g][k]);
            partial[(int64_t)b * stride + i0 + g] = t;
        }
    }
}

// V_dst = w * scale[s]
__global__ __launch_bounds__(KR_THREADS) void k_scale_to_v(const SysVec* __restrict__ sv, const int32_t* __restrict__ tile_start,
                                                           int nsys, int dst, const double* __restrict__ scale,
                                                           const int32_t* __restrict__ active) {
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    if (active && !active[s]) return;
    const SysVec V = sv[s];
    const double a = scale[s];
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
    double2* out = V.v + (int64_t)dst * V.vstride;
    const double2* src = V.w;
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        if (idx < V.len) out[idx] = cscale<double>(src[idx], a);
    }
}

// x += sum_{i<cnt} y_i Z_i
template <class TZ>
__global__ __launch_bounds__(KR_THREADS) void k_update_x(const SysVec* __restrict__ sv, const int32_t* __restrict__ tile_start,
                                                         int nsys, const int32_t* __restrict__ cnts, const double2* __restrict__ y,
                                                         int ystride) {
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    const int cnt = cnts[s];
    if (cnt <= 0) return;
    const SysVec V = sv[s];
    const double2* ys = y + (int64_t)s * ystride;
    const TZ* z = (const TZ*)V.z;
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        if (idx >= V.len) continue;
        double2 acc = V.x[idx];
        for (int i = 0; i < cnt; ++i) {
            const TZ zz = z[(int64_t)i * V.zstride + idx];
            acc = cfma<double>(ys[i], make_double2((double)zz.x, (double)zz.y), acc);
        }
        V.x[idx] = acc;
    }
}

// |vec|^2 partials; vec = w (which 0) or f (which 1)
__global__ __launch_bounds__(KR_THREADS) void k_norm_partials(const SysVec* __restrict__ sv, const int32_t* __restrict__ tile_start,
                                                              int nsys, int which, double2* __restrict__ partial,
                                                              const int32_t* __restrict__ active) {
    __shared__ double2 red[KR_THREADS / 64];
    const int b = blockIdx.x;
    const int s = tile_system(tile_start, nsys, b);
    if (active && !active[s]) return;
    const SysVec V = sv[s];
    const double2* vec = which == 0 ? V.w : V.f;
    const int64_t base = (int64_t)(b - tile_start[s]) * KR_TILE;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < PER_THREAD; ++e) {
        const int64_t idx = base + e * KR_THREADS + threadIdx.x;
        if (idx < V.len) { const double2 a = vec[idx]; acc = fma(a.x, a.x, fma(a.y, a.y, acc)); }
    }
    const double2 tot = block_sum(make_double2(acc, 0.0), red);
    if (threadIdx.x == 0) partial[b] = tot;
}

__global__ void k_norm_finish(const int32_t* __restrict__ tile_start, int nsys, const double2* __restrict__ partial,
                              double* __restrict__ out, const int32_t* __restrict__ active) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || (active && !active[s])) return;
    double acc = 0.0;
    for (int t = tile_start[s]; t < tile_start[s + 1]; ++t) acc += partial[t].x;
    out[s] = sqrt(acc);
}

// Column j of the Hessenberg matrix of every active system: H[0..j, j] holds the Gram-Schmidt
// coefficients, H[j+1, j] = ||w||.  Apply the previous rotations, form the new one, rotate g.
// Complex rotation G = [[c, s], [-conj(s), c]], c real: G (a, b)^t = (r, 0)^t.
__global__ void k_arnoldi_finish(int nsys, int j, int k, double2* __restrict__ H, double2* __restrict__ cs,
                                 double2* __restrict__ g, const double* __restrict__ nrms, double* __restrict__ inv_norm,
                                 double* __restrict__ est, const int32_t* __restrict__ active) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || (active && !active[s])) return;
    double2* Hc = H + ((int64_t)s * k + j) * (k + 1);       // column j, k+1 rows
    double2* C = cs + (int64_t)s * 2 * k;                   // C[2i] = (c, 0), C[2i+1] = s
    double2* G = g + (int64_t)s * (k + 1);
    const double nrm = nrms[s];
    Hc[j + 1] = make_double2(nrm, 0.0);
    inv_norm[s] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = 0; i < j; ++i) {
        const double c = C[2 * i].x;
        const double2 sn = C[2 * i + 1];
        const double2 a = Hc[i], bb = Hc[i + 1];
        Hc[i] = cfma<double>(sn, bb, cscale<double>(a, c));
        Hc[i + 1] = csub<double>(cscale<double>(bb, c), cconjmul<double>(sn, a));
    }
    const double2 a = Hc[j], bb = Hc[j + 1];
    double c;
    double2 sn;
    const double aa = sqrt(cabs2<double>(a)), ab = sqrt(cabs2<double>(bb));
    if (ab == 0.0) { c = 1.0; sn = make_double2(0.0, 0.0); }
    else if (aa == 0.0) { c = 0.0; sn = make_double2(1.0, 0.0); }
    else {
        const double t = hypot(aa, ab);
        c = aa / t;
        const double2 ph = cscale<double>(a, 1.0 / aa);
        sn = cscale<double>(cmul<double>(ph, make_double2(bb.x, -bb.y)), 1.0 / t);
    }
    C[2 * j] = make_double2(c, 0.0);
    C[2 * j + 1] = sn;
    Hc[j] = cfma<double>(sn, bb, cscale<double>(a, c));
    Hc[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = G[j];
    G[j + 1] = cscale<double>(cconjmul<double>(sn, gj), -1.0);
    G[j] = cscale<double>(gj, c);
    est[s] = sqrt(cabs2<double>(G[j + 1]));
}

// y = H^{-1} g, H upper triangular cnt x cnt (rotated Hessenberg)
__global__ void k_backsolve(int nsys, int k, const double2* __restrict__ H, const double2* __restrict__ g,
                            const int32_t* __restrict__ cnt, double2* __restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const int m = cnt[s];
    const double2* Hs = H + (int64_t)s * k * (k + 1);
    const double2* G = g + (int64_t)s * (k + 1);
    double2* Y = y + (int64_t)s * k;
    for (int i = m - 1; i >= 0; --i) {
        double2 acc = G[i];
        for (int l = i + 1; l < m; ++l) acc = cfms<double>(Hs[(int64_t)l * (k + 1) + i], Y[l], acc);
        const double2 d = Hs[(int64_t)i * (k + 1) + i];
        Y[i] = (d.x == 0.0 && d.y == 0.0) ? make_double2(0.0, 0.0) : cmul<double>(acc, cinv<double>(d));
    }
}

// V_0 = w / beta, g = (beta, 0, ...)
__global__ void k_start_g(int nsys, const double* __restrict__ beta, double2* __restrict__ g, int gstride,
                          double* __restrict__ inv) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    double2* G = g + (int64_t)s * gstride;
    for (int i = 0; i < gstride; ++i) G[i] = make_double2(0.0, 0.0);
    G[0] = make_double2(beta[s], 0.0);
    inv[s] = beta[s] > 0.0 ? 1.0 / beta[s] : 0.0;
}

__global__ void k_cycle_flags(int nsys, const double* __restrict__ beta, const double* __restrict__ fnorm,
                              const CycleCtl* __restrict__ ctl, const int32_t* __restrict__ it, double* __restrict__ rr,
                              int32_t* __restrict__ done, int32_t* __restrict__ active, int32_t* __restrict__ cnt) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const double f = fnorm[s];
    const double r = f > 0.0 ? beta[s] / f : 0.0;
    const int d = (r <= ctl->tol) || f == 0.0;
    rr[s] = r;
    done[s] = d;
    active[s] = !d && it[s] < ctl->maxit;
    cnt[s] = 0;
}

__global__ void k_iter_flags(int nsys, int j, const double* __restrict__ est, const double* __restrict__ fnorm,
                             const CycleCtl* __restrict__ ctl, int32_t* __restrict__ it, int32_t* __restrict__ cnt,
                             int32_t* __restrict__ active) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || !active[s]) return;
    const int i = it[s] + 1;
    it[s] = i;
    cnt[s] = j + 1;
    const double e = est[s] / fnorm[s];
    if (!(e > ctl->tol) || i >= ctl->maxit) active[s] = 0;
}

__global__ void k_zero_i32(int32_t* __restrict__ a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

// ---------------------------------------------------------------------------------------------
void launch_multidot(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j, double2* partial,
                     int stride, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, j, partial, stride, active);
}
void launch_reduce_partials(const int32_t* tile_start, int nsys, const double2* partial, int stride, int cnt, double2* h,
                            int hstride, int accumulate, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(nsys), dim3(64), 0, s, tile_start, partial, stride, cnt, h, hstride, accumulate,
                       active);
}
void launch_multiaxpy(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j, const double2* h,
                      int hstride, const int32_t* active, hipStream_t s, double2* npart) {
    hipLaunchKernelGGL(k_multiaxpy, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, j, h, hstride, active,
                       npart);
}
void launch_multiaxpy_dot(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j, const double2* h,
                          int hstride, double2* partial, int stride, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_multiaxpy_dot, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, j, h, hstride, partial,
                       stride, active);
}
void launch_scale_to_v(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int dst, const double* scale,
                       const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_to_v, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, dst, scale, active);
}
void launch_update_x(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, const int32_t* cnt,
                     const double2* y, int ystride, int zprec, hipStream_t s) {
    if (zprec == 0)
        hipLaunchKernelGGL(k_update_x<double2>, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, cnt, y, ystride);
    else
        hipLaunchKernelGGL(k_update_x<float2>, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, cnt, y, ystride);
}
void launch_arnoldi_finish(int nsys, int j, int k, double2* H, double2* cs, double2* g, const double* nrm,
                           double* inv_norm, double* est, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_arnoldi_finish, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, j, k, H, cs, g, nrm, inv_norm, est,
                       active);
}
void launch_backsolve(int nsys, int k, const double2* H, const double2* g, const int32_t* cnt, double2* y, hipStream_t s) {
    hipLaunchKernelGGL(k_backsolve, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, k, H, g, cnt, y);
}
void launch_norms(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int which, double2* partial,
                  double* out, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_partials, dim3(ntiles), dim3(KR_THREADS), 0, s, sv, tile_start, nsys, which, partial, active);
    hipLaunchKernelGGL(k_norm_finish, dim3((nsys + 63) / 64), dim3(64), 0, s, tile_start, nsys, partial, out, active);
}
void launch_norm_finish(const int32_t* tile_start, int nsys, const double2* partial, double* out, const int32_t* active,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_norm_finish, dim3((nsys + 63) / 64), dim3(64), 0, s, tile_start, nsys, partial, out, active);
}
void launch_start_cycle(int nsys, const double* beta, double* inv, double2* g, int gstride, hipStream_t s) {
    hipLaunchKernelGGL(k_start_g, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, beta, g, gstride, inv);
}
void launch_cycle_flags(int nsys, const double* beta, const double* fnorm, const CycleCtl* ctl, const int32_t* it,
                        double* rr, int32_t* done, int32_t* active, int32_t* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_flags, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, beta, fnorm, ctl, it, rr, done, active,
                       cnt);
}
void launch_iter_flags(int nsys, int j, const double* est, const double* fnorm, const CycleCtl* ctl, int32_t* it,
                       int32_t* cnt, int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_iter_flags, dim3((nsys + 63) / 64), dim3(64), 0, s, nsys, j, est, fnorm, ctl, it, cnt, active);
}
void launch_zero_i32(int32_t* a, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, s, a, n);
}

}  // namespace hs
