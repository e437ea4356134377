// Launchers of the helmsweep kernels (host side).  Every launcher enqueues on the given stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_common.h"

namespace hs {

// Offsets (in double2 elements) of the profile tables inside one problem's table block.
struct ProfileLayout {
    int32_t n, B;
    int32_t s1n, is1n, s1h, s2n, is2n, s2h, mvn, imvn, mvh, mdn, imdn, mdh, total;
    static ProfileLayout make(int n, int B) {
        ProfileLayout L{};
        L.n = n; L.B = B;
        int o = 0;
        L.s1n = o; o += n; L.is1n = o; o += n; L.s1h = o; o += n + 1;
        L.s2n = o; o += n; L.is2n = o; o += n; L.s2h = o; o += n + 1;
        L.mvn = o; o += B; L.imvn = o; o += B; L.mvh = o; o += B + 1;
        L.mdn = o; o += 2 * B - 1; L.imdn = o; o += 2 * B - 1; L.mdh = o; o += 2 * B;
        L.total = o;
        return L;
    }
};

// Operands of one problem's matvec: y = A x (f == nullptr) or y = f - A x.
struct MvDev {
    const void* x;   // complex128 or complex64 [nrhs][N]
    void* y;         // complex128 [nrhs][N]
    const void* f;   // complex128 [nrhs][N] or nullptr
    int32_t nrhs;
    int32_t sys0;    // batch system index of right-hand side 0 (for the active mask)
};

void launch_profiles(const ProfileLayout& L, double2* tab, double h, double omega, double eta_p,
                     double eta_m, double C, hipStream_t s);
void launch_inv_c2(const double* c, double* ic2, int64_t N, int* bad, hipStream_t s);
// Batched (io, blk_start device tables over nprob problems) or single problem (io == nullptr,
// blk_start == nullptr: operands io_val, problem probs[0]).  active: per-system flags indexed by
// MvDev::sys0 + right-hand side (nullptr: every right-hand side); inactive ones are skipped.
void launch_matvec(const ProbDev* probs, const MvDev* io, MvDev io_val, const int32_t* blk_start, int nprob,
                   int total_blocks, int x_prec, const int32_t* active, hipStream_t s);
int matvec_blocks(int n);

// a2: factor `nsub` strips of height `bs` (all of one problem). prec 0: complex128 store,
// 1: complex64 store.  status: device int, bit 0 set on a zero / non-finite pivot.
// Returns false if `bs` has no compiled instance.
// One launch over nsub strips of height bs (each SubDev names its problem and factor address);
// status[prob] is or-ed with 1 when a pivot of that problem is zero or not finite.
bool launch_factor(int bs, int prec, const ProbDev* probs, const SubDev* subs, int nsub, int* status, hipStream_t s);

// a3/a4: sweep chains and middle layer.
//   phase 0: forward substitution + diagonal applications along each chain
//   phase 1: backward substitution along each chain
// vec_in/vec_out precisions: 0 complex128, 1 complex64.  Factor precision `prec`.
// io: device table indexed by ChainDev::prob, or nullptr to use io_val for every chain.
// ksplit: 1 (each 16/32/64-lane row group serves its own right-hand side) or the number of row
// groups per wave (all groups serve one right-hand side, splitting each block-vector product).
// active: per-system flags indexed by ChainDev::sys0 + i (i < nq), or nullptr; a chain whose
// systems are all inactive does nothing (its outputs keep their previous contents).
bool launch_chains(int B, int prec, int in_prec, int out_prec, int phase, int ksplit, const ProbDev* probs,
                   const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill,
                   const int32_t* active, hipStream_t s);
// The same chains with two waves per chain (backward and forward pass on separate waves, one LDS
// barrier per step); strip heights up to 17.
bool launch_chains2(int B, int prec, int in_prec, int out_prec, int phase, int ksplit, const ProbDev* probs,
                    const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill,
                    const int32_t* active, hipStream_t s);
// Segmented chains (strip solves partitioned into SEG-column segments): one workgroup of `waves`
// waves per chain; ChainDev::wrhs = waves per right-hand side (ceil(segments / 4)), nq right-hand
// sides per workgroup.  io[p].prop must hold the problem's propagators (launch_prop).  Returns false
// for strip heights without an instance or a workgroup beyond the LDS.  max_n: the largest n of
// the problems in the table (sizes the shared propagator area).
// ws: workspace of seg_ws_elems(nchains, waves) complex elements of the compute precision.
// only_front != 0: the front strips (F, E) alone (the moving layers applied by the compressed chains).
bool launch_chains_seg(int B, int prec, int in_prec, int out_prec, int phase, const ProbDev* probs,
                       const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, int waves, int max_n,
                       const int32_t* active, void* ws, hipStream_t s, int only_front = 0);
int64_t seg_ws_elems(int nchains, int waves);
bool seg_supported(int B);
// LDS of a segmented workgroup of `waves` waves for problems up to max_n, and whether it fits.
size_t seg_lds_bytes(int prec, int B, int waves, int max_n);
bool seg_fits(int prec, int B, int waves, int max_n);
// Segment propagators of front strips, one wave per work item (Q segments of one strip).
bool launch_prop(int B, int prec, const ProbDev* probs, const PropDev* work, int nwork, hipStream_t s);
bool launch_middle(int B, int prec, int in_prec, int out_prec, int ksplit, const ProbDev* probs,
                   const ChainDev* mids, int nmids, const IoDev* io, IoDev io_val, void* spill,
                   const int32_t* active, hipStream_t s);
// Lanes per row group (right-hand sides per wave) for chains of strip height B and for the middle.
int chain_rhs_per_wave(int B);
int middle_rhs_per_wave(int B);
// Padded rows per right-hand side inside a wave.
int chain_padded_rows(int B);
// Workspace of one chain, in complex elements of the compute precision: the forward products of
// two strips (2 * n * 64) and a 1 KiB slot per wave that absorbs the stores of ticks without output.
constexpr int64_t kSpillPad = 128;
__host__ __device__ inline int64_t chain_spill_elems(int n) { return (int64_t)n * 64 * 2 + kSpillPad; }

// Test hook: full-input / full-output solve of one strip (complex128 vectors [nrhs][rows][n]).
bool launch_subsolve(int bs, int prec, const ProbDev* prob, const void* fac, const double2* ris2, int rstep, int cdir,
                     int jl, const void* g, void* x, int nrhs, void* spill, hipStream_t s);

// ---- FGMRES building blocks (a6), batched over systems --------------------------------------
// A "system" is one right-hand side of one problem.  Vectors of system s start at base[s] and have
// len[s] complex128 elements; tiles of KR_TILE elements, tile_start[s] = first tile of system s.
struct SysVec {
    double2* v;        // first Krylov vector V_0 of the system; V_j = v + j * vstride
    void* z;           // first preconditioned vector Z_0 (complex128 or complex64); Z_j = z + j * zstride
    double2* w;        // work vector
    double2* x;        // solution
    const double2* f;  // right-hand side
    int64_t len, vstride, zstride;
};

constexpr int KR_TILE = 2048;
constexpr int KR_THREADS = 256;

// All tile kernels skip the tiles of systems with active[s] == 0 (active may be nullptr: all active).
// partial[t * stride + i] = sum over tile t of conj(V_i) . w   for i = 0..j
void launch_multidot(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j,
                     double2* partial, int stride, const int32_t* active, hipStream_t s);
// h[s * hstride + i] (+)= sum of partial over the tiles of system s, i < cnt (active systems only)
void launch_reduce_partials(const int32_t* tile_start, int nsys, const double2* partial, int stride, int cnt,
                            double2* h, int hstride, int accumulate, const int32_t* active, hipStream_t s);
// w -= sum_{i<=j} h[s][i] V_i; npart (optional, ntiles entries): per-tile |w|^2 partial sums of the
// result, for launch_norm_finish
void launch_multiaxpy(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j,
                      const double2* h, int hstride, const int32_t* active, hipStream_t s, double2* npart = nullptr);
// Basis vectors the fused update + dot kernel keeps in registers per element (j + 1 <= KR_FUSE).
constexpr int KR_FUSE = 24;
// k_multiaxpy with h, then the dot products of the updated w with V_0..V_j into partial (as
// launch_multidot), in one pass over V; j + 1 <= KR_FUSE.
void launch_multiaxpy_dot(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int j, const double2* h,
                          int hstride, double2* partial, int stride, const int32_t* active, hipStream_t s);
// V_dst = w * scale[s]
void launch_scale_to_v(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int dst,
                       const double* scale, const int32_t* active, hipStream_t s);
// x += sum_{i<cnt[s]} y[s][i] Z_i ; zprec 0 (complex128 Z) / 1 (complex64 Z)
void launch_update_x(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, const int32_t* cnt,
                     const double2* y, int ystride, int zprec, hipStream_t s);
// ||vec|| per system, vec = w (which 0) or f (which 1); partial needs ntiles entries
void launch_norms(const SysVec* sv, const int32_t* tile_start, int nsys, int ntiles, int which,
                  double2* partial, double* out, const int32_t* active, hipStream_t s);
// out[s] = sqrt(sum of partial[t].x over the tiles of system s) (the second half of launch_norms)
void launch_norm_finish(const int32_t* tile_start, int nsys, const double2* partial, double* out, const int32_t* active,
                        hipStream_t s);
// Column j of the Hessenberg matrix H[s][j][0..k] of every active system: set H[j+1][j] = nrm[s],
// apply the previous Givens rotations, form the new one, rotate g; est[s] = |g[j+1]|,
// inv_norm[s] = 1/nrm[s] (0 if nrm == 0).
void launch_arnoldi_finish(int nsys, int j, int k, double2* H, double2* cs, double2* g, const double* nrm,
                           double* inv_norm, double* est, const int32_t* active, hipStream_t s);
// y[s] = H[s]^{-1} g[s] (upper triangular, size cnt[s])
void launch_backsolve(int nsys, int k, const double2* H, const double2* g, const int32_t* cnt, double2* y,
                      hipStream_t s);
// g[s] = (beta[s], 0, ..., 0), inv[s] = 1/beta[s] (0 if beta == 0)
void launch_start_cycle(int nsys, const double* beta, double* inv, double2* g, int gstride, hipStream_t s);

// Convergence bookkeeping on the device, for a restart cycle that runs without host round trips
// (graph replay).  tol and maxit live in device memory so that one captured cycle serves every call.
struct CycleCtl {
    double tol;
    int32_t maxit;
    int32_t pad_;
};
// Start of a cycle: rr[s] = beta[s] / fnorm[s] (0 if fnorm == 0), done[s] = rr <= tol or f == 0,
// active[s] = !done && it[s] < maxit, cnt[s] = 0.
void launch_cycle_flags(int nsys, const double* beta, const double* fnorm, const CycleCtl* ctl, const int32_t* it,
                        double* rr, int32_t* done, int32_t* active, int32_t* cnt, hipStream_t s);
// After Arnoldi step j, for every active system: it += 1, cnt = j + 1; the system leaves the cycle
// when est / fnorm <= tol (or is NaN) or it reaches maxit.
void launch_iter_flags(int nsys, int j, const double* est, const double* fnorm, const CycleCtl* ctl, int32_t* it,
                       int32_t* cnt, int32_t* active, hipStream_t s);
// a[0..n) = 0 (a kernel, so that it may sit inside a captured graph)
void launch_zero_i32(int32_t* a, int n, hipStream_t s);

// Compressed moving-layer chains (layer-row-to-layer-row strip maps, precomputed per segment of SEG
// columns): available strip heights for a segment width, complex elements of one segment's block.
bool chainc_supported(int B, int seg);
int64_t comp_block_elems(int B, int seg);
// Compressed blocks of the segments listed in `work` from the stored factors (prec 0: complex128
// factors, 1: complex64); blocks are stored in complex64.
bool launch_compress(int B, int seg, int prec, const ProbDev* probs, const CompDev* work, int nwork, hipStream_t s);
// One workgroup per chain (problem, front, up to rq right-hand sides), `waves` waves (one per segment
// of the largest problem, <= 16); io[p].cmp holds problem p's blocks.  Moving layers only: F / E and the
// middle layer are applied by the other kernels.  Returns false for unsupported shapes.
bool launch_chains_comp(int B, int seg, int rq, int in_prec, int out_prec, int phase, const ProbDev* probs,
                        const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, int waves,
                        const int32_t* active, hipStream_t s);
size_t chainc_lds_bytes(int B, int seg, int rq, int waves);

// Matrix-core chains (factor precision HELM_C64_BF16X3): one wave per chain (problem, front, up to 16
// right-hand sides), every strip of the front in the phase's order, block products in bf16x3 on
// v_mfma_f32_16x16x32_bf16.  io[p].msp holds problem p's split blocks (launch_msplit), ws a workspace
// of chainm_ws_f4(n, B) float4 per chain at chain.spill_off.  Returns false for unsupported B.
bool chainm_supported(int B);
int64_t chainm_ws_f4(int n, int B);
// Split copy of ncols stored columns (complex64 factors, B-row strips) into msp (same layout).
bool launch_msplit(int B, const void* fac, void* msp, int64_t ncols, hipStream_t s);
bool launch_chains_mfma(int B, int in_prec, int out_prec, int phase, const ProbDev* probs, const ChainDev* chains,
                        int nchains, const IoDev* io, IoDev io_val, void* ws, const int32_t* active, hipStream_t s);

// Copy of `bytes` (a multiple of width) from src to dst with width-byte loads and stores (8 or 16).
bool launch_calib_copy(const void* src, void* dst, int64_t bytes, int width, hipStream_t s);

// Device address of the allocation-free entry point's static scratch array on the current device
// (looked up once per device), or nullptr with noalloc_error() set.
void* noalloc_scratch();
const char* noalloc_error();

}  // namespace hs
