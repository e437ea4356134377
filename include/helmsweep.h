/*
 * helmsweep.h -- C-ABI of the moving-PML sweeping preconditioner for the 2D Helmholtz equation
 * on one MI355X (gfx950).
 *
 * Method: B. Engquist and L. Ying, "Sweeping preconditioner for the Helmholtz equation: moving
 * perfectly matched layers" (2010).  Problem statement (Section 1): solve
 *     Delta u + omega^2 / c(x)^2 u = f   on (0,1)^2
 * with PML absorbing layers on all four sides (eq. sigma, Section 3.1), discretised by the 5-point
 * stencil of the symmetric stretched operator (eq. helmd) on the n x n interior grid, h = 1/(n+1),
 * and preconditioned by the approximate LDL^t sweep built from moving-PML subproblems
 * (Section 2.2, Algorithms 3 and 4 with two fronts) of the shifted operator A_alpha (eq. helmalpha).
 *
 * Conventions shared by every entry point
 *   - Vectors are complex, interleaved (re, im): complex128 = two doubles, complex64 = two floats.
 *     A block of nrhs vectors is laid out [nrhs][N], N = n*n, and one vector in row-by-row order,
 *     index (j-1)*n + (i-1) for grid point (ih, jh): x1 fastest (Section 2.1).
 *   - Every data pointer is a HIP *device* pointer owned by the caller (e.g. a torch tensor); the
 *     library reads/writes it only during the call (stream-ordered) and never keeps it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All work is enqueued
 *     on it; helm_assemble, sweep_factor and fgmres_solve* synchronise it before returning, the
 *     others are asynchronous.
 *   - Handles own their device memory and are released only by the matching *_free.  A
 *     sweep_factors_t refers to its helm_problem_t, which must outlive it.  Handles are bound to
 *     the device current at creation and are not thread-safe.
 *   - Return codes: HELM_OK (0); HELM_ENOTCONV (+1, fgmres reached maxit, outputs filled with the
 *     last iterate); negative codes leave outputs untouched:
 *       HELM_EINVAL    bad argument (shape, width, non-finite or non-positive c, tol outside (0,1)),
 *       HELM_ENOMEM    size check or device allocation failed,
 *       HELM_EHIP      a HIP runtime error,
 *       HELM_ESINGULAR a zero or non-finite pivot while inverting a diagonal block.
 *     helm_last_error() returns a message for the last failing call on the calling thread.
 */
#ifndef HELMSWEEP_H
#define HELMSWEEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK 0
#define HELM_ENOTCONV 1
#define HELM_EINVAL (-1)
#define HELM_ENOMEM (-2)
#define HELM_EHIP (-3)
#define HELM_ESINGULAR (-4)

/* Precision of the stored factors and of the sweep arithmetic. */
#define HELM_C128 0        /* complex128 factors, FP64 sweep                                  */
#define HELM_C64 1         /* factors computed in FP64, stored as complex64, FP32 sweep        */
/* Factors as HELM_C64; the sweep's block products Lambda_i^{-1} [B x R] (Algorithm 4) on the matrix
 * cores in bf16x3 form (each FP32 operand split into bf16 hi + lo, three bf16 products, FP32
 * accumulation: about 2^-16 relative error per product), 16 right-hand sides per wave, the strips'
 * column recurrences as in the plain sweep; the middle layer on the FP32 vector path.  Accepted by
 * sweep_factor only (the handle then reports HELM_C64 storage); B in {4, 5, 7, 9, 13, 17}. */
#define HELM_C64_BF16X3 2

typedef struct helm_problem_s* helm_problem_t;
typedef struct sweep_factors_s* sweep_factors_t;
typedef struct helm_batch_s* helm_batch_t;

typedef struct {
    int32_t n;            /* interior points per side (N = n*n unknowns); n >= 2B+3                  */
    double omega;         /* angular frequency > 0; the wave number is omega / 2pi (Section 1)       */
    double alpha;         /* shift of the preconditioner's operator, omega^2 -> (omega + i alpha)^2
                             (eq. helmalpha); >= 0, the paper uses 2 in 2D                            */
    int32_t pml_w;        /* physical PML on every side: damped grid rows/columns, >= 1 (eq. sigma)   */
    int32_t mpml_w;       /* moving PML: damped rows of a layer subproblem, >= 1 (Section 2.2);
                             a subproblem strip has B = mpml_w + 1 rows                               */
    double pml_C;         /* PML strength C > 0 in sigma = (C/eta)((t-eta)/eta)^2 (eq. sigma)         */
    int32_t b_convention; /* 0: eta = (w+1)h, B = w+1 (default); 1: eta = w h, B = w                 */
    int32_t layers_d;     /* grid rows eliminated per sweep step (end of Section 2.3); 0 or 1 = one
                             row per step, the only form these kernels run: any other value returns
                             HELM_EINVAL                                                              */
    int32_t exact_mode;   /* 0: moving-PML subproblems (Section 2.2).  A non-zero value asks for the
                             exact Schur complements (every subproblem the whole remaining block of
                             A_alpha, Section 2.1), whose strips grow to n rows: the fixed-height strip
                             kernels cannot hold them, so it returns HELM_EINVAL (the CPU reference
                             implements that mode for testing)                                        */
} helm_params;

/* Library version string. */
const char* helm_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* helm_last_error(void);

/* a1 -- Assemble the problem (eq. sigma, eq. helmd, eq. helmalpha): validates c, computes the PML
 * stretch profiles s = (1 + i sigma/omega)^{-1} in x1 and x2 for the physical and the moving
 * layers, and 1/c^2 on the grid, in FP64 on the device.
 *   p     parameters (host pointer, read during the call)
 *   c     device, real float64 [n*n], row-by-row; copied, every value finite and > 0
 *   out   receives the new handle
 * Supported strip heights: B and 2B-1 both in {4,5,7,9,13,17,25,33} (e.g. B = 4,5,7,9,13,17). */
int helm_assemble(const helm_params* p, const double* c, void* stream, helm_problem_t* out);

/* a1 again, in place: recompute the problem's tables from a new velocity c (same n and parameters)
 * without allocating.  Same checks and synchronisation as helm_assemble. */
int helm_reassemble(helm_problem_t A, const double* c, void* stream);

/* Grid size of a problem (n) or -1 for a NULL handle. */
int helm_problem_n(helm_problem_t A);

/* a5 -- y = A x for nrhs vectors, the true operator (alpha = 0) in FP64 (eq. helmd).
 *   x  device [nrhs][N], complex128 (x_prec = HELM_C128) or complex64 (x_prec = HELM_C64)
 *   y  device [nrhs][N] complex128; must not overlap x. */
int helm_matvec(helm_problem_t A, const void* x, int32_t x_prec, void* y, int32_t nrhs, void* stream);

/* a2 -- Algorithm 3 (two-front form, Section 2.3): factor every moving-PML subproblem of A_alpha --
 * F (rows 1..B), E (rows n-B+1..n), the lower layers m = B+1..c-1 (rows m-B+1..m), the upper layers
 * m = n-B..c+1 (rows m..m+B-1) and the middle layer c (rows c-B+1..c+B-1), c = (n+1)/2 (odd n) or
 * n/2+1 (even n).  Each strip, in the x2-first ordering of Section 2.2, is block tridiagonal over the
 * n columns with B x B (middle: 2B-1) blocks D_i and diagonal couplings E_i; the block LU
 * Lambda_1 = D_1, Lambda_i = D_i - E_i Lambda_{i-1}^{-1} E_i is computed in FP64 and the complex
 * symmetric Lambda_i^{-1} stored packed (upper triangle) in `prec`.  Where the segmented sweep
 * applies (B <= 13 and n <= 1024, or n <= 512 with complex128 factors) the propagator of every
 * 16-column segment of every front strip (the product of its steps' maps, a B x B block) is formed
 * from the stored factors as well; they serve only to apply the same M_alpha with a shorter
 * sequential path.
 * With prec = HELM_C64_BF16X3 the complex64 factors are also kept split into bf16 hi / lo (the same
 * size again, F / E / moving strips) for the matrix-core sweep.
 * Returns HELM_ESINGULAR if a block has a zero or non-finite pivot.  Synchronises `stream`. */
int sweep_factor(helm_problem_t A, int32_t prec, void* stream, sweep_factors_t* out);

/* a2 again, in place: recompute every strip factor from the problem's current tables (after
 * helm_reassemble) without allocating.  Same checks and synchronisation as sweep_factor. */
int sweep_refactor(sweep_factors_t M, void* stream);

/* Bytes of device memory held by a factor handle (0 for NULL). */
int64_t sweep_factor_bytes(sweep_factors_t M);

/* a3/a4 -- u = M_alpha f (Algorithm 4, two fronts + middle): forward substitution with the diagonal
 * T~ applications, then backward substitution.  One banded solve per layer and phase.
 *   f  device [nrhs][N]; u device [nrhs][N]; vec_prec (HELM_C128 / HELM_C64) is the element type of
 *   both.  f and u must not overlap.  Asynchronous. */
int sweep_apply(sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t vec_prec, void* stream);

/* Allocation-free form of sweep_apply, for callers that cannot allocate device memory: code running
 * under HIP graph capture, allocation-free serving loops, harnesses that forbid hipMalloc.  The same
 * operation, kernels, schedule and results as sweep_apply (u = M_alpha f, same arguments); the chain
 * tables and sweep workspaces, which sweep_apply keeps in memory the handle allocates, go instead to
 * one statically allocated scratch array of HELM_NOALLOC_SCRATCH_BYTES per GPU (created when the
 * library is loaded on that GPU, held until the process ends).  No hipMalloc / hipFree or allocating
 * library call is made; the tables are copied into the scratch with hipMemcpyAsync on `stream` (a call
 * whose nrhs differs from the previous one on the same factors first synchronises `stream`).
 * Returns HELM_ENOMEM (and launches nothing) when the call needs more scratch than that, e.g. n = 511
 * with 64 right-hand sides in complex128.  Every call on one GPU shares its scratch, which keeps
 * the last call's contents (no kernel reads scratch it has not written in the same call): calls that
 * overlap on one GPU (other streams, other threads) race, so serialise them. */
#define HELM_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int sweep_apply_noalloc(sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t vec_prec, void* stream);

/* One subproblem's T~ (test hook for parity of a2): solve H_s x = g for subproblem `sub`
 * (0 = F, 1..L = lower layers B+1.., L+1 = E, L+2.. = upper layers n-B.., last = middle) with
 * g and x device complex128 [nrhs][rows][n] in the strip's local row order (local row 0 is the row
 * farthest from the layer row, F/E: rows 1.. / n.. respectively); full input, full output. */
int sweep_subsolve(sweep_factors_t M, int32_t sub, const void* g, void* x, int32_t nrhs, void* stream);

/* Number of subproblems of a factor handle and the strip height of one of them. */
int sweep_num_subproblems(sweep_factors_t M);
int sweep_subproblem_rows(sweep_factors_t M, int32_t sub);

/* a6 -- Right-preconditioned flexible GMRES(restart) on A u = f with u = M_alpha y (Section 2.3's
 * GMRES, in flexible right-preconditioned form): FP64 Arnoldi (classical Gram-Schmidt with one
 * re-orthogonalisation), FP64 matvec and residual; the preconditioner in the factors' precision.
 * Stops when the true ||f - A u||_2 / ||f||_2 <= tol for every right-hand side, or after maxit
 * iterations (HELM_ENOTCONV).
 *   f      device complex128 [nrhs][N];  u device complex128 [nrhs][N]: in x0, out the solution
 *   iters  host int32 [nrhs] (may be NULL): iterations per right-hand side
 *   relres host double [nrhs] (may be NULL): final true relative residual per right-hand side
 * Synchronises `stream`. */
int fgmres_solve(helm_problem_t A, sweep_factors_t M, const void* f, void* u, int32_t nrhs,
                 int32_t restart, double tol, int32_t maxit, int32_t* iters, double* relres,
                 void* stream);

/* a7 -- Batched form: `count` problems of possibly different n (same B and factor precision), each
 * with its own factors and nrhs[k] right-hand sides, solved together: every phase of every FGMRES
 * iteration is one launch over the whole batch.
 *   A, M, nrhs  host arrays [count]; the handles must outlive the batch */
int helm_batch_create(const helm_problem_t* A, const sweep_factors_t* M, const int32_t* nrhs,
                      int32_t count, int32_t restart, void* stream, helm_batch_t* out);

/* Solve the batch.  f[k], u[k]: device complex128 [nrhs[k]][N_k] (u[k]: x0 in, solution out).
 * iters / relres: host arrays of sum(nrhs) entries (problem-major), may be NULL. */
int fgmres_solve_batch(helm_batch_t b, const void* const* f, void* const* u, double tol,
                       int32_t maxit, int32_t* iters, double* relres, void* stream);

/* a7 -- Graph form of fgmres_solve_batch (the solver of Section 2.3 with few host round trips).
 * on != 0: later solves of the batch run every restart cycle as replays of hipGraphs captured at
 * the first such solve -- the Arnoldi steps with the preconditioner in chunks of 4, then the update,
 * the new residual and the convergence flags -- with the per-system bookkeeping (iteration counts,
 * leaving the cycle at the Arnoldi estimate, maxit) done by device kernels.  A system that converges
 * inside a cycle leaves through its flag and its kernels return at once; the host reads the flags
 * between chunks (restart/4 + 1 times per cycle instead of once per step) and skips the remaining
 * chunks of a cycle in which no system is left.  Results equal the eager form's bit for bit.  The
 * graphs are captured again after helm_batch_tune; the timing phases do not cover replays.
 * on == 0 (the default): eager launches, the host checks the estimate after every step; frees the
 * graphs.  Returns HELM_EINVAL for a NULL batch. */
int helm_batch_set_graph(helm_batch_t b, int32_t on);

/* Apply M_alpha to every right-hand side of the batch in one set of launches (f[k], u[k] as above,
 * complex128). */
int sweep_apply_batch(helm_batch_t b, const void* const* f, void* const* u, void* stream);

/* a7 -- Autotune the batch's sweep schedule: times the batched preconditioner application (on the
 * batch's own first Krylov block, zeroed) for every candidate schedule and keeps the fastest for all
 * later solves and applications of the batch.  Candidates: the segmented chains (every strip solve
 * split into 16-column segments joined by a short sequential pass over segment propagators; strip
 * heights <= 13 and n <= 1024, or 512 for complex128 factors) in workgroups of the fewest waves that
 * hold one right-hand side of the largest problem and of 2x and 4x as many where they fit the LDS
 * (several right-hand sides of a problem per workgroup), and the plain chains with two waves
 * per chain (backward and forward pass of a strip pair on separate waves, heights <= 17) or one,
 * each with the number of row groups every right-hand side's block products are split over (1, 2,
 * 4, ... dividing the row groups of a wave).  Each is run `reps` times after one warm-up.  Results
 * are unchanged up to rounding order.
 *   ksplit, waves, segmented: host (may be NULL): 1 in segmented if the segmented chains won, then
 *                             waves = their workgroup's waves and ksplit = 0; else the plain
 *                             chains' split and waves per chain
 *   ms: host (may be NULL): its time per application, milliseconds
 * Overwrites the batch's Krylov work space; synchronises `stream`. */
int helm_batch_tune(helm_batch_t b, int32_t reps, void* stream, int32_t* ksplit, int32_t* waves,
                    int32_t* segmented, double* ms);

/* a7 -- Apply a sweep schedule found earlier by helm_batch_tune (on a batch of the same problem sizes,
 * right-hand-side counts, strip height and factor precision), without timing anything: kind, ksplit
 * and waves as helm_batch_tune reports them (kind 0 plain chains: ksplit divides the right-hand-side
 * lanes of a wave, waves 1 or 2; kind 1 segmented chains: waves = their workgroup size; kind 2
 * compressed moving chains: ksplit = 4 or 8 right-hand sides per workgroup; kind 3 matrix-core chains,
 * for HELM_C64_BF16X3 factors).  Returns HELM_EINVAL if the batch cannot run that schedule (and keeps
 * its current one).  Host-side tables only; synchronous. */
int helm_batch_set_schedule(helm_batch_t b, int32_t kind, int32_t ksplit, int32_t waves);

/* a2 for the whole batch (Algorithm 3 for every problem): recompute the factors of every member
 * from its problem's current tables, all height-B strips of all problems in one launch and the
 * middle strips in a second one that overlaps it, then (segmented sweep) the segment propagators of
 * all problems in a third.  Equivalent to sweep_refactor on each member;
 * allocates nothing.  Returns HELM_ESINGULAR naming the first problem with a zero or non-finite
 * pivot.  Synchronises `stream`. */
int sweep_refactor_batch(helm_batch_t b, void* stream);

/* Per-phase kernel timing with HIP events recorded on the launch stream around every kernel
 * group (process-wide; off by default).  Phases: 0 assemble, 1 factor, 2 sweep forward chains,
 * 3 sweep middle layer, 4 sweep backward chains, 5 matvec, 6 Krylov vector kernels, 7 the front
 * strips F and E on their own (compressed chains only; otherwise inside 2 and 4).
 * helm_timing_read fills ms[8] (summed milliseconds) and launches[8] (kernel launches), waiting
 * for the recorded events; reset != 0 clears the records. */
#define HELM_NPHASES 8
int helm_timing_enable(int32_t on);
int helm_timing_read(double* ms, int64_t* launches, int32_t reset);

/* Measurement hook (row d): copy `bytes` (a multiple of `width`) from device buffer src to device
 * buffer dst (not overlapping) with loads and stores of `width` bytes per lane (8 or 16): a kernel
 * that moves exactly the bytes it is given, against which hardware traffic counters (bytes fetched
 * from and written to HBM per dispatch) are scaled.  Asynchronous; HELM_EINVAL for other widths. */
int helm_calib_copy(const void* src, void* dst, int64_t bytes, int32_t width, void* stream);

void helm_free(helm_problem_t A);
void sweep_free(sweep_factors_t M);
void helm_batch_free(helm_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* HELMSWEEP_H */
