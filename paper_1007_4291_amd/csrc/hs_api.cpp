// C-ABI of the helmsweep library: handles, argument checks, and host control of FGMRES.
// Every arithmetic step of the method runs in the HIP kernels of hs_*.hip; this file only
// validates arguments, allocates device memory, builds launch descriptors and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/helmsweep.h"
#include "hs_common.h"
#include "hs_kernels.h"

using namespace hs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(HELM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK()                                                                            \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) return fail(HELM_EHIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

// Device allocation owned by a handle.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(HELM_ENOMEM, "hipMalloc(%zu bytes): %s", b, hipGetErrorString(e));
        }
        bytes = b;
        return HELM_OK;
    }
    template <class T> T* as() const { return (T*)p; }
};

// Size pre-check: fail with HELM_ENOMEM, before any allocation, when `need` bytes exceed the device
// memory currently free (the allocations of one call would not fit).
int precheck_bytes(double need, const char* what) {
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HELM_EHIP, "hipMemGetInfo: %s", hipGetErrorString(e));
    }
    if (need > (double)fr)
        return fail(HELM_ENOMEM, "%s needs %.3g GB of device memory, %.3g GB free (of %.3g GB)", what, need * 1e-9,
                    (double)fr * 1e-9, (double)tot * 1e-9);
    return HELM_OK;
}

bool supported_B(int B) { return B == 4 || B == 5 || B == 7 || B == 9 || B == 13 || B == 17; }

constexpr int64_t kMaxN = 32767;

// Per-phase kernel timing (process-wide, off by default): a start/stop event pair around each
// kernel group, read back and summed on demand.
enum Phase { PH_ASSEMBLE = 0, PH_FACTOR, PH_SWEEP_FWD, PH_SWEEP_MID, PH_SWEEP_BWD, PH_MATVEC, PH_KRYLOV, PH_SWEEP_FRONT,
             PH_N };
struct TimerRec { int phase; int launches; hipEvent_t a, b; };
struct Timing {
    bool on = false;
    bool capturing = false;   // launches are being recorded into a graph: no events
    std::vector<TimerRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        return e;
    }
};
Timing& timing() { static Timing t; return t; }

// Records an event pair around the enclosed launches when timing is on.
struct PhaseScope {
    TimerRec rec{};
    hipStream_t s;
    bool live = false;
    PhaseScope(int phase, hipStream_t st, int launches = 1) : s(st) {
        Timing& T = timing();
        if (!T.on || T.capturing) return;
        rec.phase = phase;
        rec.launches = launches;
        rec.a = T.get();
        rec.b = T.get();
        if (!rec.a || !rec.b) return;
        live = hipEventRecord(rec.a, s) == hipSuccess;
    }
    ~PhaseScope() {
        if (!live) return;
        if (hipEventRecord(rec.b, s) == hipSuccess) timing().recs.push_back(rec);
    }
};

}  // namespace

struct helm_problem_s {
    helm_params prm{};
    int n = 0, B = 0, c = 0, L_lo = 0, L_up = 0, nsub = 0;
    double h = 0;
    ProfileLayout lay{};
    DevBuf tab, ic2, pd, flag;
    ProbDev host{};
};

// Launch plan of a single-problem application for nrhs right-hand sides (host side): the plain chain
// table (groups of Q right-hand sides per front), the middle table (Qm per wave), the segmented chain
// table where the segmented sweep applies, and the workspace sizes.
struct SoloPlan {
    std::vector<ChainDev> ch, md, sc, cc, mc;
    int ks_chain = 1, ks_mid = 1, waves = 1, seg_wg = 0, kind = 0, cwaves = 0, crq = 8;
    size_t spill_bytes = 0, segws_bytes = 0, mws_bytes = 0;
};

struct sweep_factors_s {
    helm_problem_t A = nullptr;
    int prec = 0;
    DevBuf fac, subs, spill, status;
    int64_t fac_elems = 0;
    // segmented sweep: propagators of the front strips and their work table (seg: available)
    DevBuf prop, propw;
    int npropw = 0;
    bool seg = false;
    // compressed moving-layer chains: per-segment blocks of every moving strip, their work table
    // (comp: available), segment width
    DevBuf cmp, compw;
    int ncompw = 0, cseg = 0;
    bool comp = false;
    // matrix-core chains (HELM_C64_BF16X3): split copy of the F / E / moving strips' blocks
    bool mfma = false;
    DevBuf msp;
    std::vector<SubDev> hsubs;
    std::vector<int> sub_rows;
    // single-problem chain tables (rebuilt when nrhs changes)
    DevBuf chains, mids, segch, segws, cchains, mchains, mws;
    int nmch = 0;
    int chains_nrhs = -1, nchains = 0, nmids = 0, ks_chain = 1, ks_mid = 1, waves = 1, ncch = 0, cwaves = 0, crq = 8;
    int nsegch = 0, seg_wg = 0, kind = 0;   // kind 1: segmented chains, 2: compressed moving chains, 3: matrix-core chains
    helm_batch_t solo = nullptr;    // cached batch of one for fgmres_solve
    std::unique_ptr<SoloPlan> na_plan;   // host tables of the last sweep_apply_noalloc call
    int na_nrhs = -1;
    int solo_nrhs = -1, solo_restart = -1;
    ~sweep_factors_s();
};

struct helm_batch_s {
    int count = 0, restart = 0, prec = 0, B = 0;
    std::vector<helm_problem_t> A;
    std::vector<sweep_factors_t> M;
    std::vector<int> nrhs;
    std::vector<int64_t> N;
    int nsys = 0, ntiles = 0, mv_blocks = 0, nchains = 0, nmids = 0, ks_chain = 1, ks_mid = 1, waves = 1;
    std::vector<int> sys_prob, sys_rhs;
    std::vector<int32_t> tiles_h;
    DevBuf probs, chains, mids, io_sweep, io_apply, mv_z, mv_res, mv_blk, sv, tiles;
    DevBuf V, Z, W, spill;
    DevBuf H, cs, g, y, partial, hbuf, nrm, inv, est, fnorm, beta, active, cnt;
    std::vector<int64_t> voff, zoff, woff;   // element offsets of each problem's blocks
    size_t zelem = 16;
    // batched refactorisation: strip tables of all problems (height B, and the middles) and a
    // second stream so that the two launches overlap
    DevBuf fsubs, msubs, fstatus;
    int nfsubs = 0, nmsubs = 0;
    // segmented sweep: propagator work of all problems, chain table, workgroup waves; kind 1 selects it
    DevBuf propw, segch, segws;
    int npropw = 0, nsegch = 0, seg_wg = 0, seg_maxn = 0, kind = 0;
    bool seg = false;
    // compressed moving chains (kind 2; F / E through the segmented kernel): compression work of all
    // problems, chain table (problem, front, group of crq right-hand sides), waves per workgroup
    DevBuf compw, cch;
    int ncompw = 0, ncch = 0, cwaves = 0, crq = 8, cseg = 0;
    bool comp = false;
    // matrix-core chains (kind 3, factors HELM_C64_BF16X3): chain table (problem, front, 16 right-hand
    // sides) and workspace
    DevBuf mch, mws;
    int nmch = 0;
    bool mfma = false;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // graph form of FGMRES: a restart cycle captured once (on its own stream) as a few graphs that are
    // replayed, with the convergence bookkeeping on the device: tol / maxit, iterations, final relative
    // residuals, flags.  gexec: the Arnoldi steps in chunks of kGraphChunk, then the cycle's tail.
    bool use_graph = false;
    hipStream_t gstream = nullptr;
    std::vector<hipGraphExec_t> gexec;
    DevBuf ctl, it_d, done_d, rr_d;
    void drop_graph() {
        for (hipGraphExec_t g : gexec) (void)hipGraphExecDestroy(g);
        gexec.clear();
    }
    ~helm_batch_s() {
        drop_graph();
        if (gstream) (void)hipStreamDestroy(gstream);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
};

sweep_factors_s::~sweep_factors_s() {
    if (solo) helm_batch_free(solo);
}

// ------------------------------------------------------------------------------------------------
extern "C" const char* helm_version(void) { return "helmsweep 0.1 (gfx950)"; }
extern "C" const char* helm_last_error(void) { return g_err.c_str(); }

static int check_params(const helm_params* p, int* Bout) {
    if (!p) return fail(HELM_EINVAL, "params is NULL");
    if (p->b_convention != 0 && p->b_convention != 1) return fail(HELM_EINVAL, "b_convention must be 0 or 1");
    if (p->layers_d != 0 && p->layers_d != 1)
        return fail(HELM_EINVAL, "layers_d=%d: only one grid row per sweep step (layers_d 0 or 1) is built",
                    p->layers_d);
    if (p->exact_mode != 0)
        return fail(HELM_EINVAL, "exact_mode: exact Schur complements need strips of up to n rows; the strip "
                                 "kernels hold at most 2B-1 rows");
    if (p->pml_w < 1 || p->mpml_w < 1) return fail(HELM_EINVAL, "pml_w and mpml_w must be >= 1");
    const int B = p->b_convention == 0 ? p->mpml_w + 1 : p->mpml_w;
    if (!supported_B(B)) return fail(HELM_EINVAL, "strip height B=%d not compiled (supported 4,5,7,9,13,17)", B);
    if (p->n < 2 * B + 3) return fail(HELM_EINVAL, "n=%d too small for B=%d (need n >= 2B+3)", p->n, B);
    if (p->n > kMaxN) return fail(HELM_EINVAL, "n=%d exceeds %lld", p->n, (long long)kMaxN);
    if (!(p->omega > 0.0) || !std::isfinite(p->omega)) return fail(HELM_EINVAL, "omega must be finite and > 0");
    if (!(p->alpha >= 0.0) || !std::isfinite(p->alpha)) return fail(HELM_EINVAL, "alpha must be finite and >= 0");
    if (!(p->pml_C > 0.0) || !std::isfinite(p->pml_C)) return fail(HELM_EINVAL, "pml_C must be finite and > 0");
    const int wp = p->b_convention == 0 ? p->pml_w + 1 : p->pml_w;
    if (2 * wp > p->n + 1) return fail(HELM_EINVAL, "physical PML wider than half the domain");
    *Bout = B;
    return HELM_OK;
}

// Run the a1 kernels into A's tables from velocity c and check c.
static int assemble_into(helm_problem_t A, const double* c, hipStream_t s) {
    const helm_params* p = &A->prm;
    const int n = A->n, B = A->B;
    const int64_t N = (int64_t)n * n;
    HIPCHK(hipMemsetAsync(A->flag.p, 0, sizeof(int), s));
    const double h = A->h;
    const double eta_p = (p->b_convention == 0 ? p->pml_w + 1 : p->pml_w) * h;
    const double eta_m = B * h;
    {
        PhaseScope ph(PH_ASSEMBLE, s, 2);
        launch_profiles(A->lay, A->tab.as<double2>(), h, p->omega, eta_p, eta_m, p->pml_C, s);
        LAUNCHCHK();
        launch_inv_c2(c, A->ic2.as<double>(), N, A->flag.as<int>(), s);
        LAUNCHCHK();
    }
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, A->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return fail(HELM_EINVAL, "velocity c has a non-finite or non-positive value");
    return HELM_OK;
}

extern "C" int helm_assemble(const helm_params* p, const double* c, void* stream, helm_problem_t* out) {
    int B = 0;
    int rc = check_params(p, &B);
    if (rc) return rc;
    if (!c || !out) return fail(HELM_EINVAL, "c or out is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<helm_problem_s> A(new helm_problem_s());
    A->prm = *p;
    const int n = p->n;
    A->n = n; A->B = B;
    A->c = (n % 2 == 1) ? (n + 1) / 2 : n / 2 + 1;
    A->L_lo = A->c - 1 - B;
    A->L_up = n - B - A->c;
    A->nsub = A->L_lo + A->L_up + 3;
    A->h = 1.0 / (n + 1);
    A->lay = ProfileLayout::make(n, B);
    const int64_t N = (int64_t)n * n;
    if ((rc = A->tab.alloc(sizeof(double2) * A->lay.total))) return rc;
    if ((rc = A->ic2.alloc(sizeof(double) * N))) return rc;
    if ((rc = A->flag.alloc(sizeof(int)))) return rc;
    if ((rc = A->pd.alloc(sizeof(ProbDev)))) return rc;
    if ((rc = assemble_into(A.get(), c, s))) return rc;
    const double h = A->h;
    ProbDev& P = A->host;
    P.n = n; P.B = B; P.c = A->c; P.L_lo = A->L_lo; P.L_up = A->L_up; P.nsub = A->nsub;
    P.ih2 = 1.0 / (h * h);
    const double kr = p->omega, ki = p->alpha;
    P.kappa2 = make_double2(kr * kr - ki * ki, 2.0 * kr * ki);
    P.omega2 = make_double2(kr * kr, 0.0);
    double2* t = A->tab.as<double2>();
    const ProfileLayout& L = A->lay;
    P.s1n = t + L.s1n; P.is1n = t + L.is1n; P.s1h = t + L.s1h;
    P.s2n = t + L.s2n; P.is2n = t + L.is2n; P.s2h = t + L.s2h;
    P.mvn = t + L.mvn; P.imvn = t + L.imvn; P.mvh = t + L.mvh;
    P.mdn = t + L.mdn; P.imdn = t + L.imdn; P.mdh = t + L.mdh;
    P.ic2 = A->ic2.as<double>();
    HIPCHK(hipMemcpy(A->pd.p, &P, sizeof(ProbDev), hipMemcpyHostToDevice));
    *out = A.release();
    return HELM_OK;
}

extern "C" int helm_reassemble(helm_problem_t A, const double* c, void* stream) {
    if (!A || !c) return fail(HELM_EINVAL, "NULL argument");
    return assemble_into(A, c, (hipStream_t)stream);
}

extern "C" int helm_problem_n(helm_problem_t A) { return A ? A->n : -1; }

extern "C" void helm_free(helm_problem_t A) { delete A; }

extern "C" int helm_matvec(helm_problem_t A, const void* x, int32_t x_prec, void* y, int32_t nrhs, void* stream) {
    if (!A || !x || !y) return fail(HELM_EINVAL, "NULL argument");
    if (nrhs < 0) return fail(HELM_EINVAL, "nrhs < 0");
    if (x_prec != HELM_C128 && x_prec != HELM_C64) return fail(HELM_EINVAL, "x_prec must be HELM_C128 or HELM_C64");
    if (nrhs == 0) return HELM_OK;
    MvDev mv{x, y, nullptr, nrhs, 0};
    PhaseScope ph(PH_MATVEC, (hipStream_t)stream);
    launch_matvec(A->pd.as<ProbDev>(), nullptr, mv, nullptr, 1, matvec_blocks(A->n), x_prec, nullptr,
                  (hipStream_t)stream);
    LAUNCHCHK();
    return HELM_OK;
}

// ------------------------------------------------------------------------------------------------
// a2: factorisation
// ------------------------------------------------------------------------------------------------
// Segmented sweep sizes: segments per strip, waves per right-hand side (4 segments per wave).
static int seg_count(int n) { return (n + SEG - 1) / SEG; }
static int seg_waves_rhs(int n) { return (seg_count(n) + 3) / 4; }
// Segment propagators of one strip: a row-major B x B block per segment, the strip's array rounded
// to 16 bytes (complex elements).
static int64_t seg_strip_elems(int n, int B) { return ((int64_t)seg_count(n) * B * B + 1) & ~(int64_t)1; }
// HELM_SWEEP_SEG=0 / 1 forces the plain / segmented chains; unset: segmented where available.
static int seg_env() {
    const char* e = std::getenv("HELM_SWEEP_SEG");
    return e ? std::atoi(e) : -1;
}
// Waves per segmented workgroup to aim for (HELM_SEG_WG; 0: the fewest that hold one right-hand side
// of the largest problem), halved until the workgroup fits the LDS.
static int seg_wg_target(int prec, int B, const std::vector<int>& n) {
    const char* e = std::getenv("HELM_SEG_WG");
    int t = e ? std::atoi(e) : 0;
    int wmin = 1, maxn = 1;
    for (int v : n) { wmin = std::max(wmin, (seg_count(v) + 3) / 4); maxn = std::max(maxn, v); }
    while (t > wmin && !seg_fits(prec, B, t, maxn)) t /= 2;
    return t > wmin ? t : 0;
}

// Compressed moving chains: segment width (HELM_CSEG = 16 or 32; default 32), available when the
// factors are complex64, the segmented kernel serves F / E, the strip height has an instance and a
// strip's segments fit one workgroup (one wave each, at most 16).
static int cseg_env() {
    const char* e = std::getenv("HELM_CSEG");
    const int v = e ? std::atoi(e) : 32;
    return (v == 16 || v == 32) ? v : 32;
}
static bool comp_possible(int prec, bool seg, int B, int n, int cseg) {
    return prec == HELM_C64 && seg && chainc_supported(B, cseg) && (n + cseg - 1) / cseg <= 16;
}
// HELM_SWEEP_KIND = 0 / 1 / 2 forces the plain / segmented / compressed chains for the single-problem
// path and as the batch's starting schedule (unset: the best available, compressed first).
static int kind_env() {
    const char* e = std::getenv("HELM_SWEEP_KIND");
    return e ? std::atoi(e) : -1;
}

// Run the a2 kernels for every strip of M's problem and check the pivots.
static int factor_into(sweep_factors_t M, hipStream_t s) {
    helm_problem_t A = M->A;
    const int n = A->n, B = A->B;
    HIPCHK(hipMemsetAsync(M->status.p, 0, sizeof(int), s));
    const ProbDev* pd = A->pd.as<ProbDev>();
    {
        PhaseScope ph(PH_FACTOR, s, 2 + (M->seg ? 1 : 0) + (M->comp ? 1 : 0) + (M->mfma ? 1 : 0));
        if (!launch_factor(B, M->prec, pd, M->subs.as<SubDev>(), A->nsub - 1, M->status.as<int>(), s))
            return fail(HELM_EINVAL, "no factor kernel for B=%d", B);
        LAUNCHCHK();
        if (!launch_factor(2 * B - 1, M->prec, pd, M->subs.as<SubDev>() + (A->nsub - 1), 1, M->status.as<int>(), s))
            return fail(HELM_EINVAL, "no factor kernel for middle height %d", 2 * B - 1);
        LAUNCHCHK();
        if (M->seg) {
            if (!launch_prop(B, M->prec, pd, M->propw.as<PropDev>(), M->npropw, s))
                return fail(HELM_EINVAL, "no propagator kernel for B=%d", B);
            LAUNCHCHK();
        }
        if (M->comp) {
            if (!launch_compress(B, M->cseg, M->prec == HELM_C128 ? 0 : 1, pd, M->compw.as<CompDev>(), M->ncompw, s))
                return fail(HELM_EINVAL, "no compression kernel for B=%d, segment width %d", B, M->cseg);
            LAUNCHCHK();
        }
        if (M->mfma) {
            if (!launch_msplit(B, M->fac.p, M->msp.p, (int64_t)(A->nsub - 1) * n, s))
                return fail(HELM_EINVAL, "no split kernel for B=%d", B);
            LAUNCHCHK();
        }
    }
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, M->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st & 2) return fail(HELM_EINVAL, "internal: strips of different sizes in one factor workgroup");
    if (st) return fail(HELM_ESINGULAR, "zero or non-finite pivot while inverting a diagonal block");
    return HELM_OK;
}

extern "C" int sweep_factor(helm_problem_t A, int32_t prec, void* stream, sweep_factors_t* out) {
    if (!A || !out) return fail(HELM_EINVAL, "NULL argument");
    if (prec != HELM_C128 && prec != HELM_C64 && prec != HELM_C64_BF16X3)
        return fail(HELM_EINVAL, "prec must be HELM_C128, HELM_C64 or HELM_C64_BF16X3");
    if (prec == HELM_C64_BF16X3 && !chainm_supported(A->B))
        return fail(HELM_EINVAL, "HELM_C64_BF16X3 supports strip heights B in {4, 5, 7, 9, 13, 17} (B=%d)", A->B);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<sweep_factors_s> M(new sweep_factors_s());
    M->A = A;
    M->mfma = prec == HELM_C64_BF16X3;
    if (M->mfma) prec = HELM_C64;                       // storage: complex64 (plus the split copy)
    M->prec = prec;
    const int n = A->n, B = A->B;
    // stored column length (packed block + coupling scalars, padded to 16 bytes) per precision
    const int64_t pk = prec == HELM_C128 ? col_stride<double>(B) : col_stride<float>(B);
    const int64_t pkm = prec == HELM_C128 ? col_stride<double>(2 * B - 1) : col_stride<float>(2 * B - 1);
    M->fac_elems = (int64_t)(A->nsub - 1) * n * pk + (int64_t)n * pkm;
    const size_t esz = prec == HELM_C128 ? sizeof(double2) : sizeof(float2);
    int rc;
    {
        // factor store plus, for the segmented sweep, one B x B propagator per 16 columns of every strip
        const double props = (double)esz * (double)(A->nsub - 1) * (double)(((n + SEG - 1) / SEG) * B * B + 1);
        if ((rc = precheck_bytes((double)esz * (double)M->fac_elems + props, "the factor store"))) return rc;
    }
    if ((rc = M->fac.alloc(esz * (size_t)M->fac_elems))) return rc;
    if (M->mfma) {
        const double mb = (double)sizeof(float2) * (double)(A->nsub - 1) * n * pk;
        if ((rc = precheck_bytes(mb, "the split copy of the factors"))) return rc;
        if ((rc = M->msp.alloc((size_t)mb))) return rc;
    }
    // strip descriptors: F, lower layers, E, upper layers (all height B), then the middle (2B-1).
    // Consecutive layers of a front alternate their column direction; jprev / jnext are the layer
    // rows before and after each layer in its front's sweep (the middle row after the last one).
    auto& S = M->hsubs;
    S.clear();
    const int c = A->c;
    for (int t = 0; t <= A->L_lo; ++t) {
        const int jl = B + t;
        S.push_back(SubDev{0, t == 0 ? SUB_PHYS : SUB_MOVE, jl - (B - 1), 1, (t & 1) ? -1 : 1, jl,
                           t >= 1 ? jl - 1 : 0, t < A->L_lo ? jl + 1 : c, (int64_t)S.size() * n * pk});
    }
    for (int t = 0; t <= A->L_up; ++t) {
        const int jl = n + 1 - B - t;
        S.push_back(SubDev{0, t == 0 ? SUB_PHYS : SUB_MOVE, jl + (B - 1), -1, (t & 1) ? -1 : 1, jl,
                           t >= 1 ? jl + 1 : 0, t < A->L_up ? jl - 1 : c, (int64_t)S.size() * n * pk});
    }
    S.push_back(SubDev{0, SUB_MID, c - B + 1, 1, 1, c, c - 1, c + 1, (int64_t)S.size() * n * pk});
    // resolve each strip's x2 profile to plain pointers into the problem's profile tables
    const ProbDev& P = A->host;
    for (SubDev& d : S) {
        if (d.kind == SUB_PHYS) {
            const int i0 = d.j0 - 1;                         // 0-based physical row of local row 0
            d.rs2 = P.s2n + i0; d.ris2 = P.is2n + i0; d.rstep = d.dir;
            // half rows: s2h[j-1] lies below row j and s2h[j] above it (in the +x2 direction)
            d.rlo = d.dir > 0 ? P.s2h + i0 : P.s2h + i0 + 1;
            d.rhi = d.dir > 0 ? P.s2h + i0 + 1 : P.s2h + i0;
        } else if (d.kind == SUB_MOVE) {
            d.rs2 = P.mvn; d.ris2 = P.imvn; d.rlo = P.mvh; d.rhi = P.mvh + 1; d.rstep = 1;
        } else {
            d.rs2 = P.mdn; d.ris2 = P.imdn; d.rlo = P.mdh; d.rhi = P.mdh + 1; d.rstep = 1;
        }
        d.facp = (char*)M->fac.p + esz * d.fac_off;
    }
    M->sub_rows.assign(S.size(), B);
    M->sub_rows.back() = 2 * B - 1;
    if ((int)S.size() != A->nsub) return fail(HELM_EINVAL, "internal: subproblem count");
    if ((rc = M->subs.alloc(sizeof(SubDev) * S.size()))) return rc;
    if ((rc = M->status.alloc(sizeof(int)))) return rc;
    HIPCHK(hipMemcpy(M->subs.p, S.data(), sizeof(SubDev) * S.size(), hipMemcpyHostToDevice));
    // segmented sweep: propagators of every segment of every front strip (not the middle)
    M->seg = !M->mfma && seg_fits(prec == HELM_C128 ? 0 : 1, B, seg_waves_rhs(n), n);
    if (M->seg) {
        const int Sg = seg_count(n);
        const int64_t per_strip = seg_strip_elems(n, B);
        if ((rc = M->prop.alloc(esz * (size_t)per_strip * (size_t)(A->nsub - 1)))) return rc;
        std::vector<PropDev> pw;
        for (int u = 0; u + 1 < A->nsub; ++u)
            for (int g = 0; g * 4 < Sg; ++g)
                pw.push_back(PropDev{0, S[u].cdir, S[u].rstep, g * 4, S[u].facp, S[u].ris2,
                                     (char*)M->prop.p + esz * (size_t)(u * per_strip)});
        if ((rc = M->propw.alloc(sizeof(PropDev) * pw.size()))) return rc;
        HIPCHK(hipMemcpy(M->propw.p, pw.data(), sizeof(PropDev) * pw.size(), hipMemcpyHostToDevice));
        M->npropw = (int)pw.size();
    }
    // compressed moving chains: one block per physical segment of every moving strip, strips in the
    // order lower front (layers B+1 .. c-1), upper front (n-B .. c+1)
    M->cseg = cseg_env();
    M->comp = comp_possible(prec, M->seg, B, n, M->cseg);
    if (M->comp) {
        const int Sg = (n + M->cseg - 1) / M->cseg;
        const int64_t blk = comp_block_elems(B, M->cseg);
        const int nmov = A->L_lo + A->L_up;
        if ((rc = precheck_bytes((double)sizeof(float2) * (double)blk * Sg * nmov, "the compressed strip blocks")))
            return rc;
        if ((rc = M->cmp.alloc(sizeof(float2) * (size_t)blk * Sg * nmov))) return rc;
        std::vector<CompDev> cw;
        for (int u = 0; u + 1 < A->nsub; ++u) {
            if (u == 0 || u == A->L_lo + 1) continue;                 // F and E
            const int k = u <= A->L_lo ? u - 1 : A->L_lo + (u - A->L_lo - 2);
            for (int sg = 0; sg < Sg; ++sg)
                cw.push_back(CompDev{0, S[u].cdir, S[u].rstep, sg, S[u].facp, S[u].ris2,
                                     (char*)M->cmp.p + sizeof(float2) * (size_t)blk * ((size_t)k * Sg + sg)});
        }
        if ((rc = M->compw.alloc(sizeof(CompDev) * std::max<size_t>(1, cw.size())))) return rc;
        if (!cw.empty())
            HIPCHK(hipMemcpy(M->compw.p, cw.data(), sizeof(CompDev) * cw.size(), hipMemcpyHostToDevice));
        M->ncompw = (int)cw.size();
    }
    if ((rc = factor_into(M.get(), s))) return rc;
    *out = M.release();
    return HELM_OK;
}

extern "C" int sweep_refactor(sweep_factors_t M, void* stream) {
    if (!M) return fail(HELM_EINVAL, "NULL argument");
    return factor_into(M, (hipStream_t)stream);
}

extern "C" int64_t sweep_factor_bytes(sweep_factors_t M) { return M ? (int64_t)M->fac.bytes : 0; }
extern "C" int sweep_num_subproblems(sweep_factors_t M) { return M ? (int)M->hsubs.size() : -1; }
extern "C" int sweep_subproblem_rows(sweep_factors_t M, int32_t sub) {
    if (!M || sub < 0 || sub >= (int)M->sub_rows.size()) return -1;
    return M->sub_rows[sub];
}

extern "C" void sweep_free(sweep_factors_t M) { delete M; }

static size_t compute_elem(int prec) { return prec == HELM_C128 ? sizeof(double2) : sizeof(float2); }

// Right-hand sides per wave and the k-split of a launch: with a single right-hand side per problem
// every row group of a wave works on it (split block-vector products); otherwise one right-hand
// side per row group.
// Right-hand sides per sweep wave: a wave has q row groups; with a k-split of ks groups per
// right-hand side it serves q / ks right-hand sides, each row-dot product split ks ways.  A single
// right-hand side always takes the full split.  HELM_SWEEP_KSPLIT (1, 2, 4, ...) overrides the
// choice for chains with several right-hand sides (values that do not divide q are ignored).
static int ksplit_override() {
    const char* e = std::getenv("HELM_SWEEP_KSPLIT");
    return e ? std::atoi(e) : 0;
}
// Waves per sweep chain: 2 (backward and forward pass on separate waves) unless HELM_SWEEP_WAVES=1.
static bool two_wave_chains(int B) {
    const char* e = std::getenv("HELM_SWEEP_WAVES");
    return B <= 17 && !(e && std::atoi(e) == 1);
}
static bool run_chains(int waves, int B, int prec, int in_prec, int out_prec, int phase, int ks, const ProbDev* probs,
                       const ChainDev* chains, int nchains, const IoDev* io, IoDev io_val, void* spill,
                       const int32_t* active, hipStream_t s) {
    if (waves == 2 && B <= 17)
        return launch_chains2(B, prec, in_prec, out_prec, phase, ks, probs, chains, nchains, io, io_val, spill, active, s);
    return launch_chains(B, prec, in_prec, out_prec, phase, ks, probs, chains, nchains, io, io_val, spill, active, s);
}

static void rhs_grouping(int B, int max_nrhs, int* Q, int* ks, int* Qm, int* ksm) {
    const int q = chain_rhs_per_wave(B), qm = middle_rhs_per_wave(B);
    const int ov = ksplit_override();
    // measured on the batched uneven workload: two groups per right-hand side beat one and four
    *ks = max_nrhs == 1 ? q : std::min(2, q);
    *ksm = max_nrhs == 1 ? qm : std::min(2, qm);
    if (max_nrhs > 1 && ov >= 1) {
        if (q % ov == 0) *ks = ov;
        if (qm % ov == 0) *ksm = ov;
    }
    *Q = q / *ks;
    *Qm = qm / *ksm;
}

// Segmented chain table: every workgroup has wg waves; problem p (largest first) gives each
// right-hand side seg_waves_rhs(n_p) of them, wg / that right-hand sides per workgroup and front.
// Workgroups are dealt to the 8 XCDs round-robin by index, so the table is laid out per XCD: all
// workgroups of one (problem, front) -- which read the same factor columns and propagators at about
// the same time -- get indices of one residue mod 8 and share that XCD's L2.  (problem, front) groups
// go, largest first, to the XCD with the least work so far; shorter XCD queues are padded with
// entries of no right-hand side (nq = 0), which return at once.  HELM_SEG_XCD=0 keeps the plain order.
constexpr int kXcds = 8;
static std::vector<ChainDev> seg_table(const std::vector<int>& n, const std::vector<int>& nrhs, int target, int* wg) {
    const int count = (int)n.size();
    int w = 1;
    for (int p = 0; p < count; ++p) w = std::max(w, seg_waves_rhs(n[p]));
    w = std::max(w, target);
    std::vector<int> order(count), base(count + 1, 0);
    for (int p = 0; p < count; ++p) { order[p] = p; base[p + 1] = base[p] + nrhs[p]; }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return n[a] > n[c]; });
    std::vector<std::vector<ChainDev>> groups;
    std::vector<double> work;
    for (int p : order) {
        const int wr = seg_waves_rhs(n[p]), R = std::max(1, w / wr);
        for (int f = 0; f < 2; ++f) {
            std::vector<ChainDev> g;
            for (int k = 0; k * R < nrhs[p]; ++k)
                g.push_back(ChainDev{p, f, k * R, std::min(R, nrhs[p] - k * R), base[p] + k * R, wr, 0});
            groups.push_back(g);
            work.push_back((double)n[p] * n[p] * (double)g.size());
        }
    }
    *wg = w;
    const char* e = std::getenv("HELM_SEG_XCD");
    std::vector<ChainDev> ch;
    if (e && std::atoi(e) == 0) {
        for (auto& g : groups) ch.insert(ch.end(), g.begin(), g.end());
        return ch;
    }
    std::vector<std::vector<ChainDev>> q(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (size_t i = 0; i < groups.size(); ++i) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        q[x].insert(q[x].end(), groups[i].begin(), groups[i].end());
        load[x] += work[i];
    }
    size_t len = 0;
    for (auto& v : q) len = std::max(len, v.size());
    for (size_t i = 0; i < len; ++i)
        for (int x = 0; x < kXcds; ++x)
            ch.push_back(i < q[x].size() ? q[x][i] : ChainDev{0, 0, 0, 0, 0, 1, 0});
    return ch;
}

// Right-hand sides per compressed-chain workgroup (HELM_CRQ = 4 or 8; default 4).
static int crq_env() {
    const char* e = std::getenv("HELM_CRQ");
    return (e && std::atoi(e) == 8) ? 8 : 4;
}
// The group size to use for `waves` segments: 8 only where its LDS fits one workgroup.
static int fit_crq(int B, int cseg, int waves, int want) {
    return (want == 8 && chainc_lds_bytes(B, cseg, 8, std::max(waves, 4)) <= 160 * 1024) ? 8 : 4;
}

// Chain kernel kind: HELM_SWEEP_SEG = 0 / 1 forces the plain / segmented chains, HELM_SWEEP_KIND = 0 / 1 /
// 2 the plain / segmented / compressed ones; unset, the compressed chains where available, else the
// segmented ones, else the plain ones.  A forced kind that is not available falls back the same way.
static int pick_kind(bool seg, bool comp) {
    const int se = seg_env();
    int k = se >= 0 ? (se == 0 ? 0 : 1) : kind_env();
    if (k < 0) k = 2;
    if (k == 2 && !comp) k = 1;
    if (k == 1 && !seg) k = 0;
    return k;
}

static SoloPlan solo_plan(const sweep_factors_t M, int nrhs) {
    SoloPlan P;
    helm_problem_t A = M->A;
    const int n = A->n, B = A->B;
    int Q, Qm;
    rhs_grouping(B, nrhs, &Q, &P.ks_chain, &Qm, &P.ks_mid);
    P.waves = two_wave_chains(B) ? 2 : 1;
    const int groups = (nrhs + Q - 1) / Q, mgroups = (nrhs + Qm - 1) / Qm;
    const int64_t per = chain_spill_elems(n);
    P.spill_bytes = compute_elem(M->prec) * (size_t)per * (size_t)std::max(2 * groups, mgroups);
    for (int g = 0; g < groups; ++g)
        for (int f = 0; f < 2; ++f)
            P.ch.push_back(ChainDev{0, f, g * Q, std::min(Q, nrhs - g * Q), g * Q, 0, (int64_t)P.ch.size() * per});
    for (int g = 0; g < mgroups; ++g)
        P.md.push_back(ChainDev{0, 0, g * Qm, std::min(Qm, nrhs - g * Qm), g * Qm, 0, (int64_t)g * per});
    if (M->seg) {
        P.sc = seg_table({n}, {nrhs}, seg_wg_target(M->prec == HELM_C128 ? 0 : 1, B, {n}), &P.seg_wg);
        P.segws_bytes = compute_elem(M->prec) * (size_t)seg_ws_elems((int)P.sc.size(), P.seg_wg);
    }
    if (M->comp) {
        P.cwaves = (n + M->cseg - 1) / M->cseg;
        P.crq = fit_crq(B, M->cseg, P.cwaves, crq_env());
        for (int g = 0; g * P.crq < nrhs; ++g)
            for (int f = 0; f < 2; ++f)
                P.cc.push_back(ChainDev{0, f, g * P.crq, std::min(P.crq, nrhs - g * P.crq), g * P.crq, 0, 0});
    }
    P.kind = pick_kind(M->seg, M->comp);
    if (M->mfma) {
        // matrix-core chains: one wave per (front, 16 right-hand sides), each with its own workspace
        const int64_t per4 = chainm_ws_f4(n, B);
        for (int g = 0; g * 16 < nrhs; ++g)
            for (int f = 0; f < 2; ++f)
                P.mc.push_back(ChainDev{0, f, g * 16, std::min(16, nrhs - g * 16), g * 16, 0, (int64_t)P.mc.size() * per4});
        P.mws_bytes = sizeof(float) * 4 * (size_t)per4 * P.mc.size();
        P.kind = 3;
    }
    return P;
}

// Single-problem chain tables and workspaces of the factor handle, (re)built when nrhs changes.
static int ensure_solo_chains(sweep_factors_t M, int nrhs, hipStream_t s) {
    const SoloPlan P = solo_plan(M, nrhs);
    M->ks_chain = P.ks_chain;
    M->ks_mid = P.ks_mid;
    M->waves = P.waves;
    int rc;
    if (M->spill.bytes < P.spill_bytes) {
        HIPCHK(hipStreamSynchronize(s));
        if ((rc = M->spill.alloc(P.spill_bytes))) return rc;
    }
    if (M->chains_nrhs == nrhs) return HELM_OK;
    HIPCHK(hipStreamSynchronize(s));
    if ((rc = M->chains.alloc(sizeof(ChainDev) * P.ch.size()))) return rc;
    if ((rc = M->mids.alloc(sizeof(ChainDev) * P.md.size()))) return rc;
    HIPCHK(hipMemcpy(M->chains.p, P.ch.data(), sizeof(ChainDev) * P.ch.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(M->mids.p, P.md.data(), sizeof(ChainDev) * P.md.size(), hipMemcpyHostToDevice));
    M->nchains = (int)P.ch.size();
    M->nmids = (int)P.md.size();
    if (M->seg) {
        if ((rc = M->segch.alloc(sizeof(ChainDev) * P.sc.size()))) return rc;
        HIPCHK(hipMemcpy(M->segch.p, P.sc.data(), sizeof(ChainDev) * P.sc.size(), hipMemcpyHostToDevice));
        M->nsegch = (int)P.sc.size();
        M->seg_wg = P.seg_wg;
        if (M->segws.bytes < P.segws_bytes && (rc = M->segws.alloc(P.segws_bytes))) return rc;
    }
    if (M->comp) {
        if ((rc = M->cchains.alloc(sizeof(ChainDev) * P.cc.size()))) return rc;
        HIPCHK(hipMemcpy(M->cchains.p, P.cc.data(), sizeof(ChainDev) * P.cc.size(), hipMemcpyHostToDevice));
        M->ncch = (int)P.cc.size();
        M->cwaves = P.cwaves;
        M->crq = P.crq;
    }
    if (M->mfma) {
        if ((rc = M->mchains.alloc(sizeof(ChainDev) * P.mc.size()))) return rc;
        HIPCHK(hipMemcpy(M->mchains.p, P.mc.data(), sizeof(ChainDev) * P.mc.size(), hipMemcpyHostToDevice));
        M->nmch = (int)P.mc.size();
        if (M->mws.bytes < P.mws_bytes) {
            if ((rc = precheck_bytes((double)P.mws_bytes, "the matrix-core chains' workspace"))) return rc;
            if ((rc = M->mws.alloc(P.mws_bytes))) return rc;
        }
    }
    M->kind = P.kind;
    M->chains_nrhs = nrhs;
    return HELM_OK;
}

// Device operands of one single-problem application: tables and workspaces.
struct SoloDev {
    const ChainDev *ch, *md, *sc, *cc;
    int nch, nmd, nsc, ncc, ks_chain, ks_mid, waves, seg_wg, kind, cwaves, crq;
    void *spill, *segws;
    const ChainDev* mc = nullptr;
    int nmc = 0;
    void* mws = nullptr;
};

static int solo_launch(const sweep_factors_t M, const SoloDev& D, const void* f, void* u, int vec_prec, hipStream_t s) {
    const ProbDev* pd = M->A->pd.as<ProbDev>();
    IoDev io{f, u, M->fac.p, M->prop.p, M->cmp.p, M->msp.p};
    const int B = M->A->B;
    if (D.kind == 2) {
        PhaseScope ph(PH_SWEEP_FRONT, s);
        if (!launch_chains_seg(B, M->prec, vec_prec, vec_prec, 0, pd, D.sc, D.nsc, nullptr, io, D.seg_wg, M->A->n, nullptr,
                               D.segws, s, 1))
            return fail(HELM_EINVAL, "no front-strip kernel for B=%d", B);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_FWD, s);
        bool ok;
        if (D.kind == 3)
            ok = launch_chains_mfma(B, vec_prec, vec_prec, 0, pd, D.mc, D.nmc, nullptr, io, D.mws, nullptr, s);
        else if (D.kind == 2)
            ok = launch_chains_comp(B, M->cseg, D.crq, vec_prec, vec_prec, 0, pd, D.cc, D.ncc, nullptr, io, D.cwaves,
                                    nullptr, s);
        else if (D.kind == 1)
            ok = launch_chains_seg(B, M->prec, vec_prec, vec_prec, 0, pd, D.sc, D.nsc, nullptr, io, D.seg_wg, M->A->n,
                                   nullptr, D.segws, s);
        else
            ok = run_chains(D.waves, B, M->prec, vec_prec, vec_prec, 0, D.ks_chain, pd, D.ch, D.nch, nullptr, io, D.spill,
                            nullptr, s);
        if (!ok) return fail(HELM_EINVAL, "no sweep kernel for B=%d (kind %d)", B, D.kind);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_MID, s);
        if (!launch_middle(B, M->prec, vec_prec, vec_prec, D.ks_mid, pd, D.md, D.nmd, nullptr, io, D.spill, nullptr, s))
            return fail(HELM_EINVAL, "no middle-strip kernel for height %d (factor precision %d, vectors %d)", 2 * B - 1,
                        M->prec, vec_prec);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_BWD, s);
        bool ok;
        if (D.kind == 3)
            ok = launch_chains_mfma(B, vec_prec, vec_prec, 1, pd, D.mc, D.nmc, nullptr, io, D.mws, nullptr, s);
        else if (D.kind == 2)
            ok = launch_chains_comp(B, M->cseg, D.crq, vec_prec, vec_prec, 1, pd, D.cc, D.ncc, nullptr, io, D.cwaves,
                                    nullptr, s);
        else if (D.kind == 1)
            ok = launch_chains_seg(B, M->prec, vec_prec, vec_prec, 1, pd, D.sc, D.nsc, nullptr, io, D.seg_wg, M->A->n,
                                   nullptr, D.segws, s);
        else
            ok = run_chains(D.waves, B, M->prec, vec_prec, vec_prec, 1, D.ks_chain, pd, D.ch, D.nch, nullptr, io, D.spill,
                            nullptr, s);
        if (!ok)
            return fail(HELM_EINVAL, "no backward sweep kernel for B=%d (factor precision %d, vectors %d, kind %d)", B,
                        M->prec, vec_prec, D.kind);
        LAUNCHCHK();
    }
    if (D.kind == 2) {
        PhaseScope ph(PH_SWEEP_FRONT, s);
        if (!launch_chains_seg(B, M->prec, vec_prec, vec_prec, 1, pd, D.sc, D.nsc, nullptr, io, D.seg_wg, M->A->n, nullptr,
                               D.segws, s, 1))
            return fail(HELM_EINVAL, "no front-strip kernel for B=%d", B);
        LAUNCHCHK();
    }
    return HELM_OK;
}

static int check_apply_args(sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t vec_prec) {
    if (!M || !f || !u) return fail(HELM_EINVAL, "NULL argument");
    if (nrhs < 0) return fail(HELM_EINVAL, "nrhs < 0");
    if (vec_prec != HELM_C128 && vec_prec != HELM_C64) return fail(HELM_EINVAL, "vec_prec must be HELM_C128 or HELM_C64");
    if (M->prec == HELM_C128 && vec_prec != HELM_C128) return fail(HELM_EINVAL, "complex128 factors need complex128 vectors");
    return HELM_OK;
}

extern "C" int sweep_apply(sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t vec_prec, void* stream) {
    int rc = check_apply_args(M, f, u, nrhs, vec_prec);
    if (rc || nrhs == 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ensure_solo_chains(M, nrhs, s))) return rc;
    const SoloDev D{M->chains.as<ChainDev>(), M->mids.as<ChainDev>(), M->segch.as<ChainDev>(), M->cchains.as<ChainDev>(),
                    M->nchains, M->nmids, M->nsegch, M->ncch, M->ks_chain, M->ks_mid, M->waves, M->seg_wg, M->kind,
                    M->cwaves, M->crq, M->spill.p, M->segws.p, M->mchains.as<ChainDev>(), M->nmch, M->mws.p};
    return solo_launch(M, D, f, u, vec_prec, s);
}

extern "C" int sweep_apply_noalloc(sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t vec_prec,
                                   void* stream) {
    int rc = check_apply_args(M, f, u, nrhs, vec_prec);
    if (rc || nrhs == 0) return rc;
    hipStream_t s = (hipStream_t)stream;
    // The plan is host data kept in the handle, so that the asynchronous copies below read memory that
    // outlives the call.  It changes only with nrhs; the stream's earlier copies from the old plan are
    // waited for before it is replaced.
    if (!M->na_plan || M->na_nrhs != nrhs) {
        if (M->na_plan) HIPCHK(hipStreamSynchronize(s));
        M->na_plan.reset(new SoloPlan(solo_plan(M, nrhs)));
        M->na_nrhs = nrhs;
    }
    const SoloPlan& P = *M->na_plan;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_ch = 0, o_md = o_ch + up(sizeof(ChainDev) * P.ch.size()), o_sc = o_md + up(sizeof(ChainDev) * P.md.size()),
                 o_cc = o_sc + up(sizeof(ChainDev) * P.sc.size()), o_sp = o_cc + up(sizeof(ChainDev) * P.cc.size()),
                 o_ws = o_sp + up(P.spill_bytes), o_mc = o_ws + up(P.segws_bytes),
                 o_mw = o_mc + up(sizeof(ChainDev) * P.mc.size()), total = o_mw + up(P.mws_bytes);
    if (total > (size_t)HELM_NOALLOC_SCRATCH_BYTES)
        return fail(HELM_ENOMEM, "sweep_apply_noalloc: n=%d with %d right-hand sides needs %zu bytes of scratch, the "
                                 "static scratch holds %d", M->A->n, nrhs, total, (int)HELM_NOALLOC_SCRATCH_BYTES);
    char* base = (char*)noalloc_scratch();
    if (!base) return fail(HELM_EHIP, "sweep_apply_noalloc: %s", noalloc_error());
    HIPCHK(hipMemcpyAsync(base + o_ch, P.ch.data(), sizeof(ChainDev) * P.ch.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(base + o_md, P.md.data(), sizeof(ChainDev) * P.md.size(), hipMemcpyHostToDevice, s));
    if (!P.sc.empty())
        HIPCHK(hipMemcpyAsync(base + o_sc, P.sc.data(), sizeof(ChainDev) * P.sc.size(), hipMemcpyHostToDevice, s));
    if (!P.cc.empty())
        HIPCHK(hipMemcpyAsync(base + o_cc, P.cc.data(), sizeof(ChainDev) * P.cc.size(), hipMemcpyHostToDevice, s));
    if (!P.mc.empty())
        HIPCHK(hipMemcpyAsync(base + o_mc, P.mc.data(), sizeof(ChainDev) * P.mc.size(), hipMemcpyHostToDevice, s));
    const SoloDev D{(const ChainDev*)(base + o_ch), (const ChainDev*)(base + o_md), (const ChainDev*)(base + o_sc),
                    (const ChainDev*)(base + o_cc), (int)P.ch.size(), (int)P.md.size(), (int)P.sc.size(),
                    (int)P.cc.size(), P.ks_chain, P.ks_mid, P.waves, P.seg_wg, P.kind, P.cwaves, P.crq, base + o_sp,
                    base + o_ws, (const ChainDev*)(base + o_mc), (int)P.mc.size(), base + o_mw};
    return solo_launch(M, D, f, u, vec_prec, s);
}

extern "C" int sweep_subsolve(sweep_factors_t M, int32_t sub, const void* g, void* x, int32_t nrhs, void* stream) {
    if (!M || !g || !x) return fail(HELM_EINVAL, "NULL argument");
    if (sub < 0 || sub >= (int)M->hsubs.size()) return fail(HELM_EINVAL, "subproblem index out of range");
    if (nrhs <= 0) return nrhs == 0 ? HELM_OK : fail(HELM_EINVAL, "nrhs < 0");
    hipStream_t s = (hipStream_t)stream;
    const int bs = M->sub_rows[sub];
    const int Q = 64 / chain_padded_rows(bs);
    const int groups = (nrhs + Q - 1) / Q;
    const size_t need = compute_elem(M->prec) * (size_t)chain_spill_elems(M->A->n) * groups;
    int rc;
    if (M->spill.bytes < need) {
        HIPCHK(hipStreamSynchronize(s));
        if ((rc = M->spill.alloc(need))) return rc;
    }
    const SubDev& S = M->hsubs[sub];
    const size_t esz = M->prec == HELM_C128 ? sizeof(double2) : sizeof(float2);
    const char* fac = (const char*)M->fac.p + esz * S.fac_off;
    if (!launch_subsolve(bs, M->prec, M->A->pd.as<ProbDev>(), fac, S.ris2, S.rstep, S.cdir, S.jl, g, x, nrhs,
                         M->spill.p, s))
        return fail(HELM_EINVAL, "no strip kernel for height %d", bs);
    LAUNCHCHK();
    return HELM_OK;
}

// ------------------------------------------------------------------------------------------------
// a6 / a7: batched FGMRES
// ------------------------------------------------------------------------------------------------
// Segmented chain table of a batch for a workgroup-size target (0: the fewest waves that hold one
// right-hand side of its largest problem), and its workspace (reallocated only to grow).  Clears
// b->seg when the workgroup does not fit.
static int build_seg_table(helm_batch_t b, int target) {
    b->drop_graph();   // a captured cycle holds the old table
    std::vector<int> nv(b->count);
    for (int p = 0; p < b->count; ++p) nv[p] = b->A[p]->n;
    int wg = 0;
    const std::vector<ChainDev> sc = seg_table(nv, b->nrhs, target, &wg);
    if (!seg_fits(b->prec == HELM_C128 ? 0 : 1, b->B, wg, b->seg_maxn)) {
        b->seg = false;
        return HELM_OK;
    }
    int rc;
    if ((rc = b->segch.alloc(sizeof(ChainDev) * sc.size()))) return rc;
    HIPCHK(hipMemcpy(b->segch.p, sc.data(), sizeof(ChainDev) * sc.size(), hipMemcpyHostToDevice));
    b->nsegch = (int)sc.size();
    b->seg_wg = wg;
    const size_t wsb = compute_elem(b->prec) * (size_t)seg_ws_elems(b->nsegch, wg);
    if (b->segws.bytes < wsb && (rc = b->segws.alloc(wsb))) return rc;
    return HELM_OK;
}

// Chain and middle tables of a batch for a given k-split (right-hand sides per wave = row groups per
// wave / k-split): problem-fronts in decreasing n, right-hand-side groups of each, and their
// workspaces.  Reallocates the workspace only when it has to grow.
static int build_chain_tables(helm_batch_t b, int ks, int ksm) {
    const int B = b->B, count = b->count;
    b->drop_graph();   // a captured cycle holds the old tables and schedule
    const int Q = chain_rhs_per_wave(B) / ks, Qm = middle_rhs_per_wave(B) / ksm;
    std::vector<int> order(count);
    for (int p = 0; p < count; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->A[a]->n > b->A[c]->n; });
    std::vector<int> base(count + 1, 0);      // first system index of each problem
    for (int p = 0; p < count; ++p) base[p + 1] = base[p] + b->nrhs[p];
    std::vector<ChainDev> ch, md;
    int64_t so = 0;
    for (int p : order)
        for (int g = 0; g * Q < b->nrhs[p]; ++g)
            for (int f = 0; f < 2; ++f) {
                ch.push_back(ChainDev{p, f, g * Q, std::min(Q, b->nrhs[p] - g * Q), base[p] + g * Q, 0, so});
                so += chain_spill_elems(b->A[p]->n);
            }
    int64_t mo = 0;
    for (int p : order)
        for (int g = 0; g * Qm < b->nrhs[p]; ++g) {
            md.push_back(ChainDev{p, 0, g * Qm, std::min(Qm, b->nrhs[p] - g * Qm), base[p] + g * Qm, 0, mo});
            mo += chain_spill_elems(b->A[p]->n);
        }
    int rc;
    if ((rc = b->chains.alloc(sizeof(ChainDev) * ch.size()))) return rc;
    if ((rc = b->mids.alloc(sizeof(ChainDev) * md.size()))) return rc;
    HIPCHK(hipMemcpy(b->chains.p, ch.data(), sizeof(ChainDev) * ch.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->mids.p, md.data(), sizeof(ChainDev) * md.size(), hipMemcpyHostToDevice));
    const size_t need = compute_elem(b->prec) * (size_t)std::max(so, mo);
    if (b->spill.bytes < need && (rc = b->spill.alloc(need))) return rc;
    b->nchains = (int)ch.size();
    b->nmids = (int)md.size();
    b->ks_chain = ks;
    b->ks_mid = ksm;
    return HELM_OK;
}

// Compressed chain table of a batch: one workgroup per (problem, front, group of crq right-hand sides),
// problems in decreasing n (the longest chains start first); waves = segments of the largest problem.
static int build_comp_table(helm_batch_t b, int crq) {
    b->drop_graph();
    const int count = b->count;
    std::vector<int> order(count), base(count + 1, 0);
    for (int p = 0; p < count; ++p) { order[p] = p; base[p + 1] = base[p] + b->nrhs[p]; }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->A[a]->n > b->A[c]->n; });
    std::vector<ChainDev> cc;
    int w = 1;
    for (int p : order) w = std::max(w, (b->A[p]->n + b->cseg - 1) / b->cseg);
    crq = fit_crq(b->B, b->cseg, w, crq);
    for (int p : order) {
        for (int g = 0; g * crq < b->nrhs[p]; ++g)
            for (int f = 0; f < 2; ++f)
                cc.push_back(ChainDev{p, f, g * crq, std::min(crq, b->nrhs[p] - g * crq), base[p] + g * crq, 0, 0});
    }
    int rc;
    if ((rc = b->cch.alloc(sizeof(ChainDev) * cc.size()))) return rc;
    HIPCHK(hipMemcpy(b->cch.p, cc.data(), sizeof(ChainDev) * cc.size(), hipMemcpyHostToDevice));
    b->ncch = (int)cc.size();
    b->cwaves = w;
    b->crq = crq;
    return HELM_OK;
}

extern "C" int helm_batch_create(const helm_problem_t* A, const sweep_factors_t* M, const int32_t* nrhs, int32_t count,
                                 int32_t restart, void* stream, helm_batch_t* out) {
    if (!A || !M || !nrhs || !out) return fail(HELM_EINVAL, "NULL argument");
    if (count <= 0) return fail(HELM_EINVAL, "count must be > 0");
    if (restart < 1 || restart > 256) return fail(HELM_EINVAL, "restart must be in [1, 256]");
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<helm_batch_s> b(new helm_batch_s());
    b->count = count;
    b->restart = restart;
    for (int k = 0; k < count; ++k) {
        if (!A[k] || !M[k]) return fail(HELM_EINVAL, "NULL handle at %d", k);
        if (M[k]->A != A[k]) return fail(HELM_EINVAL, "factors %d do not belong to problem %d", k, k);
        if (nrhs[k] < 1) return fail(HELM_EINVAL, "nrhs[%d] must be >= 1", k);
        if (k > 0 && (A[k]->B != A[0]->B || M[k]->prec != M[0]->prec || M[k]->mfma != M[0]->mfma))
            return fail(HELM_EINVAL, "batch members must share B and factor precision");
        b->A.push_back(A[k]);
        b->M.push_back(M[k]);
        b->nrhs.push_back(nrhs[k]);
        b->N.push_back((int64_t)A[k]->n * A[k]->n);
    }
    b->prec = M[0]->prec;
    b->B = A[0]->B;
    const int kk = restart, B = b->B;
    b->zelem = b->prec == HELM_C128 ? sizeof(double2) : sizeof(float2);
    // vector storage: V [k+1][R][N], Z [k][R][N], W [R][N] per problem
    int64_t vo = 0, zo = 0, wo = 0;
    for (int p = 0; p < count; ++p) {
        b->voff.push_back(vo); b->zoff.push_back(zo); b->woff.push_back(wo);
        vo += (int64_t)(kk + 1) * b->nrhs[p] * b->N[p];
        zo += (int64_t)kk * b->nrhs[p] * b->N[p];
        wo += (int64_t)b->nrhs[p] * b->N[p];
    }
    int rc;
    if ((rc = precheck_bytes((double)sizeof(double2) * (double)(vo + wo) + (double)b->zelem * (double)zo,
                             "the Krylov basis of the batch (V, Z, W)")))
        return rc;
    if ((rc = b->V.alloc(sizeof(double2) * vo))) return rc;
    if ((rc = b->Z.alloc(b->zelem * zo))) return rc;
    if ((rc = b->W.alloc(sizeof(double2) * wo))) return rc;
    // problems table
    std::vector<ProbDev> pdv;
    for (int p = 0; p < count; ++p) pdv.push_back(A[p]->host);
    if ((rc = b->probs.alloc(sizeof(ProbDev) * count))) return rc;
    HIPCHK(hipMemcpy(b->probs.p, pdv.data(), sizeof(ProbDev) * count, hipMemcpyHostToDevice));
    // strip tables for the batched refactorisation (largest problems first)
    {
        std::vector<int> ord(count);
        for (int p = 0; p < count; ++p) ord[p] = p;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return A[a]->n > A[c]->n; });
        // One factor workgroup holds Q strips that must share n: strips are ordered by n and each
        // run of equal n is padded to whole workgroups with entries that store nothing.
        std::vector<SubDev> fs, ms;
        const int qf = 64 / chain_padded_rows(B), qm = 64 / chain_padded_rows(2 * B - 1);
        auto pad = [](std::vector<SubDev>& v, int q) {
            while (v.size() % q) { v.push_back(v.back()); v.back().facp = nullptr; }
        };
        for (size_t t = 0; t < ord.size(); ++t) {
            const int p = ord[t];
            const std::vector<SubDev>& hs = M[p]->hsubs;
            for (size_t u = 0; u + 1 < hs.size(); ++u) { fs.push_back(hs[u]); fs.back().prob = p; }
            ms.push_back(hs.back());
            ms.back().prob = p;
            if (t + 1 == ord.size() || A[ord[t + 1]]->n != A[p]->n) { pad(fs, qf); pad(ms, qm); }
        }
        b->nfsubs = (int)fs.size();
        b->nmsubs = (int)ms.size();
        if ((rc = b->fsubs.alloc(sizeof(SubDev) * fs.size()))) return rc;
        if ((rc = b->msubs.alloc(sizeof(SubDev) * ms.size()))) return rc;
        if ((rc = b->fstatus.alloc(sizeof(int) * count))) return rc;
        HIPCHK(hipMemcpy(b->fsubs.p, fs.data(), sizeof(SubDev) * fs.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->msubs.p, ms.data(), sizeof(SubDev) * ms.size(), hipMemcpyHostToDevice));
        HIPCHK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    }
    // chains (longest first), middles
    b->waves = two_wave_chains(B) ? 2 : 1;
    {
        int Q, Qm, ks, ksm;
        rhs_grouping(B, *std::max_element(b->nrhs.begin(), b->nrhs.end()), &Q, &ks, &Qm, &ksm);
        if ((rc = build_chain_tables(b.get(), ks, ksm))) return rc;
    }
    // segmented chains and the propagator work of all problems
    b->seg = true;
    for (int p = 0; p < count; ++p) b->seg = b->seg && M[p]->seg;
    if (b->seg) {
        std::vector<int> nv(count);
        for (int p = 0; p < count; ++p) nv[p] = A[p]->n;
        b->seg_maxn = *std::max_element(nv.begin(), nv.end());
        if ((rc = build_seg_table(b.get(), seg_wg_target(b->prec == HELM_C128 ? 0 : 1, B, nv)))) return rc;
        if (b->seg) {
            std::vector<PropDev> pw;
            for (int p = 0; p < count; ++p) {
                std::vector<PropDev> one(M[p]->npropw);
                HIPCHK(hipMemcpy(one.data(), M[p]->propw.p, sizeof(PropDev) * one.size(), hipMemcpyDeviceToHost));
                for (PropDev& d : one) { d.prob = p; pw.push_back(d); }
            }
            if ((rc = b->propw.alloc(sizeof(PropDev) * pw.size()))) return rc;
            HIPCHK(hipMemcpy(b->propw.p, pw.data(), sizeof(PropDev) * pw.size(), hipMemcpyHostToDevice));
            b->npropw = (int)pw.size();
        }
    }
    // compressed moving chains: every member compressed with the same segment width
    b->comp = b->seg;
    b->cseg = M[0]->cseg;
    for (int p = 0; p < count; ++p) b->comp = b->comp && M[p]->comp && M[p]->cseg == b->cseg;
    if (b->comp) {
        std::vector<CompDev> cw;
        for (int p = 0; p < count; ++p) {
            std::vector<CompDev> one(M[p]->ncompw);
            if (!one.empty())
                HIPCHK(hipMemcpy(one.data(), M[p]->compw.p, sizeof(CompDev) * one.size(), hipMemcpyDeviceToHost));
            for (CompDev& d : one) { d.prob = p; cw.push_back(d); }
        }
        if ((rc = b->compw.alloc(sizeof(CompDev) * std::max<size_t>(1, cw.size())))) return rc;
        if (!cw.empty())
            HIPCHK(hipMemcpy(b->compw.p, cw.data(), sizeof(CompDev) * cw.size(), hipMemcpyHostToDevice));
        b->ncompw = (int)cw.size();
        if ((rc = build_comp_table(b.get(), crq_env()))) return rc;
    }
    b->kind = pick_kind(b->seg, b->comp);
    // matrix-core chains (HELM_C64_BF16X3 factors): one wave per (problem, front, 16 right-hand sides),
    // longest problems first, each with its own workspace
    b->mfma = M[0]->mfma;
    if (b->mfma) {
        std::vector<int> order(count), base(count + 1, 0);
        for (int p = 0; p < count; ++p) { order[p] = p; base[p + 1] = base[p] + b->nrhs[p]; }
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return A[a]->n > A[c]->n; });
        std::vector<ChainDev> mc;
        int64_t off = 0;
        for (int p : order)
            for (int g = 0; g * 16 < b->nrhs[p]; ++g)
                for (int f = 0; f < 2; ++f) {
                    mc.push_back(ChainDev{p, f, g * 16, std::min(16, b->nrhs[p] - g * 16), base[p] + g * 16, 0, off});
                    off += chainm_ws_f4(A[p]->n, B);
                }
        if ((rc = precheck_bytes((double)sizeof(float) * 4 * (double)off, "the matrix-core chains' workspace"))) return rc;
        if ((rc = b->mws.alloc(sizeof(float) * 4 * (size_t)off))) return rc;
        if ((rc = b->mch.alloc(sizeof(ChainDev) * mc.size()))) return rc;
        HIPCHK(hipMemcpy(b->mch.p, mc.data(), sizeof(ChainDev) * mc.size(), hipMemcpyHostToDevice));
        b->nmch = (int)mc.size();
        b->kind = 3;
    }
    // io tables for V_j -> Z_j, and matvec tables Z_j -> W
    std::vector<IoDev> ios((size_t)kk * count);
    std::vector<MvDev> mvz((size_t)kk * count);
    double2* V = b->V.as<double2>();
    char* Z = b->Z.as<char>();
    double2* W = b->W.as<double2>();
    std::vector<int> sys0(count, 0);
    for (int p = 1; p < count; ++p) sys0[p] = sys0[p - 1] + b->nrhs[p - 1];
    for (int j = 0; j < kk; ++j)
        for (int p = 0; p < count; ++p) {
            const int64_t blk = (int64_t)b->nrhs[p] * b->N[p];
            ios[(size_t)j * count + p] =
                IoDev{V + b->voff[p] + j * blk, Z + b->zelem * (b->zoff[p] + j * blk), M[p]->fac.p, M[p]->prop.p,
                      M[p]->cmp.p, M[p]->msp.p};
            mvz[(size_t)j * count + p] = MvDev{Z + b->zelem * (b->zoff[p] + j * blk), W + b->woff[p], nullptr, b->nrhs[p],
                                                  sys0[p]};
        }
    if ((rc = b->io_sweep.alloc(sizeof(IoDev) * ios.size()))) return rc;
    if ((rc = b->mv_z.alloc(sizeof(MvDev) * mvz.size()))) return rc;
    if ((rc = b->io_apply.alloc(sizeof(IoDev) * count))) return rc;
    if ((rc = b->mv_res.alloc(sizeof(MvDev) * count))) return rc;
    HIPCHK(hipMemcpy(b->io_sweep.p, ios.data(), sizeof(IoDev) * ios.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->mv_z.p, mvz.data(), sizeof(MvDev) * mvz.size(), hipMemcpyHostToDevice));
    std::vector<int32_t> blk(count + 1);
    int tot = 0;
    for (int p = 0; p < count; ++p) { blk[p] = tot; tot += matvec_blocks(A[p]->n); }
    blk[count] = tot;
    b->mv_blocks = tot;
    if ((rc = b->mv_blk.alloc(sizeof(int32_t) * (count + 1)))) return rc;
    HIPCHK(hipMemcpy(b->mv_blk.p, blk.data(), sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice));
    // systems and tiles
    for (int p = 0; p < count; ++p)
        for (int q = 0; q < b->nrhs[p]; ++q) { b->sys_prob.push_back(p); b->sys_rhs.push_back(q); }
    b->nsys = (int)b->sys_prob.size();
    int nt = 0;
    for (int sidx = 0; sidx < b->nsys; ++sidx) {
        b->tiles_h.push_back(nt);
        nt += (int)((b->N[b->sys_prob[sidx]] + KR_TILE - 1) / KR_TILE);
    }
    b->tiles_h.push_back(nt);
    b->ntiles = nt;
    const int ns = b->nsys;
    if ((rc = b->tiles.alloc(sizeof(int32_t) * (ns + 1)))) return rc;
    HIPCHK(hipMemcpy(b->tiles.p, b->tiles_h.data(), sizeof(int32_t) * (ns + 1), hipMemcpyHostToDevice));
    if ((rc = b->sv.alloc(sizeof(SysVec) * ns))) return rc;
    if ((rc = b->H.alloc(sizeof(double2) * (size_t)ns * kk * (kk + 1)))) return rc;
    if ((rc = b->cs.alloc(sizeof(double2) * (size_t)ns * 2 * kk))) return rc;
    if ((rc = b->g.alloc(sizeof(double2) * (size_t)ns * (kk + 1)))) return rc;
    if ((rc = b->y.alloc(sizeof(double2) * (size_t)ns * kk))) return rc;
    if ((rc = b->partial.alloc(sizeof(double2) * (size_t)nt * (kk + 1)))) return rc;
    if ((rc = b->hbuf.alloc(sizeof(double2) * (size_t)ns * (kk + 1)))) return rc;
    for (DevBuf* d : {&b->nrm, &b->inv, &b->est, &b->fnorm, &b->beta})
        if ((rc = d->alloc(sizeof(double) * ns))) return rc;
    if ((rc = b->active.alloc(sizeof(int32_t) * ns))) return rc;
    if ((rc = b->cnt.alloc(sizeof(int32_t) * ns))) return rc;
    if ((rc = b->it_d.alloc(sizeof(int32_t) * ns))) return rc;
    if ((rc = b->done_d.alloc(sizeof(int32_t) * ns))) return rc;
    if ((rc = b->rr_d.alloc(sizeof(double) * ns))) return rc;
    if ((rc = b->ctl.alloc(sizeof(CycleCtl)))) return rc;
    (void)s;
    *out = b.release();
    return HELM_OK;
}

extern "C" int sweep_refactor_batch(helm_batch_t b, void* stream) {
    if (!b) return fail(HELM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int B = b->B;
    HIPCHK(hipMemsetAsync(b->fstatus.p, 0, sizeof(int) * b->count, s));
    {
        PhaseScope ph(PH_FACTOR, s, 2 + (b->seg ? 1 : 0) + (b->comp ? 1 : 0) + (b->mfma ? b->count : 0));
        // middles (few, long) on the side stream, overlapping the many height-B strips
        HIPCHK(hipEventRecord(b->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(b->side, b->ev_fork, 0));
        if (!launch_factor(2 * B - 1, b->prec, b->probs.as<ProbDev>(), b->msubs.as<SubDev>(), b->nmsubs,
                           b->fstatus.as<int>(), b->side))
            return fail(HELM_EINVAL, "no factor kernel for middle height %d", 2 * B - 1);
        LAUNCHCHK();
        HIPCHK(hipEventRecord(b->ev_join, b->side));
        if (!launch_factor(B, b->prec, b->probs.as<ProbDev>(), b->fsubs.as<SubDev>(), b->nfsubs, b->fstatus.as<int>(), s))
            return fail(HELM_EINVAL, "no factor kernel for B=%d", B);
        LAUNCHCHK();
        if (b->seg) {
            if (!launch_prop(B, b->prec, b->probs.as<ProbDev>(), b->propw.as<PropDev>(), b->npropw, s))
                return fail(HELM_EINVAL, "no propagator kernel for B=%d", B);
            LAUNCHCHK();
        }
        if (b->comp) {
            if (!launch_compress(B, b->cseg, b->prec == HELM_C128 ? 0 : 1, b->probs.as<ProbDev>(), b->compw.as<CompDev>(),
                                 b->ncompw, s))
                return fail(HELM_EINVAL, "no compression kernel for B=%d", B);
            LAUNCHCHK();
        }
        if (b->mfma) {
            for (int p = 0; p < b->count; ++p) {
                if (!launch_msplit(B, b->M[p]->fac.p, b->M[p]->msp.p, (int64_t)(b->A[p]->nsub - 1) * b->A[p]->n, s))
                    return fail(HELM_EINVAL, "no split kernel for B=%d", B);
                LAUNCHCHK();
            }
        }
        HIPCHK(hipStreamWaitEvent(s, b->ev_join, 0));
    }
    std::vector<int> st(b->count, 0);
    HIPCHK(hipMemcpyAsync(st.data(), b->fstatus.p, sizeof(int) * b->count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int p = 0; p < b->count; ++p) {
        if (st[p] & 2) return fail(HELM_EINVAL, "internal: strips of different sizes in one factor workgroup");
        if (st[p]) return fail(HELM_ESINGULAR, "problem %d: zero or non-finite pivot while inverting a diagonal block", p);
    }
    return HELM_OK;
}

extern "C" void helm_batch_free(helm_batch_t b) { delete b; }

extern "C" int helm_timing_enable(int32_t on) {
    timing().on = on != 0;
    return HELM_OK;
}

extern "C" int helm_timing_read(double* ms, int64_t* launches, int32_t reset) {
    Timing& T = timing();
    std::vector<double> acc(PH_N, 0.0);
    std::vector<int64_t> cnt(PH_N, 0);
    for (const TimerRec& r : T.recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float e = 0.f;
        HIPCHK(hipEventElapsedTime(&e, r.a, r.b));
        acc[r.phase] += e;
        cnt[r.phase] += r.launches;
    }
    for (int i = 0; i < PH_N; ++i) {
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    if (reset) {
        for (const TimerRec& r : T.recs) { T.pool.push_back(r.a); T.pool.push_back(r.b); }
        T.recs.clear();
    }
    return HELM_OK;
}

// Enqueue M_alpha on the batch: io table `io` (device, one entry per problem), in complex128,
// out complex128 or complex64 (the factor precision for FGMRES directions).  active: per-system
// device flags (nullptr: all); chains and middles whose systems are all inactive are skipped.
static int batch_sweep(helm_batch_t b, const IoDev* io, int out_prec, const int32_t* active, hipStream_t s) {
    const ProbDev* pd = b->probs.as<ProbDev>();
    const IoDev none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (b->kind == 2) {
        PhaseScope ph(PH_SWEEP_FRONT, s);
        if (!launch_chains_seg(b->B, b->prec, 0, out_prec, 0, pd, b->segch.as<ChainDev>(), b->nsegch, io, none, b->seg_wg,
                               b->seg_maxn, active, b->segws.p, s, 1))
            return fail(HELM_EINVAL, "no front-strip kernel for B=%d", b->B);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_FWD, s);
        bool ok;
        if (b->kind == 3)
            ok = launch_chains_mfma(b->B, 0, out_prec, 0, pd, b->mch.as<ChainDev>(), b->nmch, io, none, b->mws.p, active, s);
        else if (b->kind == 2)
            ok = launch_chains_comp(b->B, b->cseg, b->crq, 0, out_prec, 0, pd, b->cch.as<ChainDev>(), b->ncch, io, none,
                                    b->cwaves, active, s);
        else if (b->kind == 1)
            ok = launch_chains_seg(b->B, b->prec, 0, out_prec, 0, pd, b->segch.as<ChainDev>(), b->nsegch, io, none,
                                   b->seg_wg, b->seg_maxn, active, b->segws.p, s);
        else
            ok = run_chains(b->waves, b->B, b->prec, 0, out_prec, 0, b->ks_chain, pd, b->chains.as<ChainDev>(), b->nchains,
                            io, none, b->spill.p, active, s);
        if (!ok) return fail(HELM_EINVAL, "no sweep kernel for B=%d / precision (kind %d)", b->B, b->kind);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_MID, s);
        if (!launch_middle(b->B, b->prec, 0, out_prec, b->ks_mid, pd, b->mids.as<ChainDev>(), b->nmids, io, none,
                           b->spill.p, active, s))
            return fail(HELM_EINVAL, "no middle-strip kernel for height %d (factor precision %d)", 2 * b->B - 1, b->prec);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_SWEEP_BWD, s);
        bool ok;
        if (b->kind == 3)
            ok = launch_chains_mfma(b->B, 0, out_prec, 1, pd, b->mch.as<ChainDev>(), b->nmch, io, none, b->mws.p, active, s);
        else if (b->kind == 2)
            ok = launch_chains_comp(b->B, b->cseg, b->crq, 0, out_prec, 1, pd, b->cch.as<ChainDev>(), b->ncch, io, none,
                                    b->cwaves, active, s);
        else if (b->kind == 1)
            ok = launch_chains_seg(b->B, b->prec, 0, out_prec, 1, pd, b->segch.as<ChainDev>(), b->nsegch, io, none,
                                   b->seg_wg, b->seg_maxn, active, b->segws.p, s);
        else
            ok = run_chains(b->waves, b->B, b->prec, 0, out_prec, 1, b->ks_chain, pd, b->chains.as<ChainDev>(), b->nchains,
                            io, none, b->spill.p, active, s);
        if (!ok)
            return fail(HELM_EINVAL, "no backward sweep kernel for B=%d (factor precision %d, kind %d)", b->B, b->prec,
                        b->kind);
        LAUNCHCHK();
    }
    if (b->kind == 2) {
        PhaseScope ph(PH_SWEEP_FRONT, s);
        if (!launch_chains_seg(b->B, b->prec, 0, out_prec, 1, pd, b->segch.as<ChainDev>(), b->nsegch, io, none, b->seg_wg,
                               b->seg_maxn, active, b->segws.p, s, 1))
            return fail(HELM_EINVAL, "no front-strip kernel for B=%d", b->B);
        LAUNCHCHK();
    }
    return HELM_OK;
}

extern "C" int helm_batch_tune(helm_batch_t b, int32_t reps, void* stream, int32_t* ksplit, int32_t* waves,
                               int32_t* segmented, double* ms) {
    if (!b) return fail(HELM_EINVAL, "NULL argument");
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    const int B = b->B, q = chain_rhs_per_wave(B);
    const int ksm = b->ks_mid;
    b->drop_graph();
    const int zprec = b->prec == HELM_C128 ? 0 : 1;
    // input: the first Krylov block of every problem, zeroed (timing does not depend on the values)
    for (int p = 0; p < b->count; ++p)
        HIPCHK(hipMemsetAsync(b->V.as<double2>() + b->voff[p], 0, sizeof(double2) * b->nrhs[p] * b->N[p], s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best_ks = b->ks_chain, best_w = b->waves, best_kind = b->kind, best_segt = 0, rc = HELM_OK;
    double best = 1e300;
    auto time_one = [&](double* per) -> int {
        const IoDev* io = b->io_sweep.as<IoDev>();
        int r = batch_sweep(b, io, zprec, nullptr, s);   // warm-up
        if (r) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(HELM_EHIP, "event record");
        for (int k = 0; k < reps && r == HELM_OK; ++k) r = batch_sweep(b, io, zprec, nullptr, s);
        if (r) return r;
        float t = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return fail(HELM_EHIP, "event timing");
        *per = (double)t / reps;
        return HELM_OK;
    };
    if (b->mfma) {
        // HELM_C64_BF16X3 factors: the matrix-core chains are the schedule; time them
        b->kind = 3;
        double per = 0;
        rc = time_one(&per);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        if (ksplit) *ksplit = 16;
        if (waves) *waves = 1;
        if (segmented) *segmented = 3;
        if (ms) *ms = per;
        return HELM_OK;
    }
    if (b->seg) {
        // segmented chains with workgroups of the fewest waves that hold one right-hand side of the
        // largest problem, and of 2x and 4x as many (several right-hand sides per workgroup) where they fit
        const int prec01 = b->prec == HELM_C128 ? 0 : 1;
        int wmin = 1;
        for (int p = 0; p < b->count; ++p) wmin = std::max(wmin, seg_waves_rhs(b->A[p]->n));
        b->kind = 1;
        for (int t : {0, 2 * wmin, 4 * wmin}) {
            if (t && !seg_fits(prec01, B, t, b->seg_maxn)) continue;
            if ((rc = build_seg_table(b, t))) break;
            double per = 0;
            if ((rc = time_one(&per))) break;
            if (per < best) { best = per; best_kind = 1; best_segt = t; }
        }
    }
    int best_crq = b->crq;
    if (b->comp && rc == HELM_OK) {
        // compressed moving chains (F / E on the segmented kernel with its minimal workgroups) with 8 or 4
        // right-hand sides per workgroup
        if ((rc = build_seg_table(b, 0)) == HELM_OK) {
            b->kind = 2;
            for (int crq : {8, 4}) {
                if ((rc = build_comp_table(b, crq))) break;
                if (b->crq != crq) continue;                  // 8 does not fit the workgroup's LDS
                double per = 0;
                if ((rc = time_one(&per))) break;
                if (per < best) { best = per; best_kind = 2; best_crq = crq; best_segt = 0; }
            }
        }
    }
    b->kind = 0;
    for (int w = (B <= 17 ? 2 : 1); w >= 1 && rc == HELM_OK; --w)
        for (int ks = 1; ks <= q && rc == HELM_OK; ks *= 2) {
            if (q % ks) continue;
            if ((rc = build_chain_tables(b, ks, ksm))) break;
            b->waves = w;
            double per = 0;
            if ((rc = time_one(&per))) break;
            if (per < best) { best = per; best_ks = ks; best_w = w; best_kind = 0; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = build_chain_tables(b, best_ks, ksm))) return rc;
    if (b->seg && (rc = build_seg_table(b, best_kind == 1 ? best_segt : 0))) return rc;
    if (b->comp && (rc = build_comp_table(b, best_crq))) return rc;
    b->waves = best_w;
    b->kind = best_kind;
    if (ksplit) *ksplit = best_kind == 0 ? best_ks : (best_kind == 2 ? best_crq : 0);
    if (waves) *waves = best_kind == 1 ? b->seg_wg : (best_kind == 2 ? b->cwaves : best_w);
    if (segmented) *segmented = best_kind;
    if (ms) *ms = best;
    return HELM_OK;
}

extern "C" int helm_calib_copy(const void* src, void* dst, int64_t bytes, int32_t width, void* stream) {
    if (!src || !dst) return fail(HELM_EINVAL, "NULL argument");
    if ((width != 8 && width != 16) || bytes < 0 || bytes % width)
        return fail(HELM_EINVAL, "width must be 8 or 16 and divide bytes");
    if (!launch_calib_copy(src, dst, bytes, width, (hipStream_t)stream)) return fail(HELM_EINVAL, "width %d", width);
    LAUNCHCHK();
    return HELM_OK;
}

extern "C" int helm_batch_set_schedule(helm_batch_t b, int32_t kind, int32_t ksplit, int32_t waves) {
    if (!b) return fail(HELM_EINVAL, "NULL argument");
    const int q = chain_rhs_per_wave(b->B);
    int rc = HELM_OK;
    switch (kind) {
        case 0:
            if (ksplit < 1 || ksplit > q || q % ksplit || waves < 1 || waves > (b->B <= 17 ? 2 : 1))
                return fail(HELM_EINVAL, "plain chains: ksplit %d / waves %d not available for B=%d", ksplit, waves, b->B);
            if ((rc = build_chain_tables(b, ksplit, b->ks_mid))) return rc;
            b->waves = waves;
            break;
        case 1:
            if (!b->seg) return fail(HELM_EINVAL, "segmented chains not available for this batch");
            if (!seg_fits(b->prec == HELM_C128 ? 0 : 1, b->B, waves, b->seg_maxn))
                return fail(HELM_EINVAL, "segmented chains: %d waves per workgroup do not fit", waves);
            if ((rc = build_seg_table(b, waves))) return rc;
            break;
        case 2:
            if (!b->comp) return fail(HELM_EINVAL, "compressed chains not available for this batch");
            if (ksplit != 4 && ksplit != 8) return fail(HELM_EINVAL, "compressed chains: ksplit must be 4 or 8");
            if ((rc = build_seg_table(b, 0))) return rc;
            if ((rc = build_comp_table(b, ksplit))) return rc;
            if (b->crq != ksplit) return fail(HELM_EINVAL, "compressed chains: %d right-hand sides do not fit", ksplit);
            break;
        case 3:
            if (!b->mfma) return fail(HELM_EINVAL, "matrix-core chains need HELM_C64_BF16X3 factors");
            b->drop_graph();
            break;
        default:
            return fail(HELM_EINVAL, "unknown schedule kind %d", kind);
    }
    b->kind = kind;
    return HELM_OK;
}

extern "C" int sweep_apply_batch(helm_batch_t b, const void* const* f, void* const* u, void* stream) {
    if (!b || !f || !u) return fail(HELM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<IoDev> io(b->count);
    for (int p = 0; p < b->count; ++p) {
        if (!f[p] || !u[p]) return fail(HELM_EINVAL, "NULL vector for problem %d", p);
        io[p] = IoDev{f[p], u[p], b->M[p]->fac.p, b->M[p]->prop.p, b->M[p]->cmp.p, b->M[p]->msp.p};
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(b->io_apply.p, io.data(), sizeof(IoDev) * b->count, hipMemcpyHostToDevice));
    return batch_sweep(b, b->io_apply.as<IoDev>(), 0, nullptr, s);
}

// r = f - A u into W and beta = ||r|| for every system of the batch (vector tables set per call).
static int batch_residual(helm_batch_t b, hipStream_t s) {
    const MvDev none{nullptr, nullptr, nullptr, 0, 0};
    {
        PhaseScope ph(PH_MATVEC, s);
        launch_matvec(b->probs.as<ProbDev>(), b->mv_res.as<MvDev>(), none, b->mv_blk.as<int32_t>(), b->count,
                      b->mv_blocks, 0, nullptr, s);
        LAUNCHCHK();
    }
    {
        PhaseScope ph(PH_KRYLOV, s, 2);
        launch_norms(b->sv.as<SysVec>(), b->tiles.as<int32_t>(), b->nsys, b->ntiles, 0, b->partial.as<double2>(),
                     b->beta.as<double>(), nullptr, s);
        LAUNCHCHK();
    }
    return HELM_OK;
}

// Arnoldi step j of the systems flagged in b->active: Z_j = M V_j, W = A Z_j, classical Gram-Schmidt
// twice against V_0..V_j, Givens update of the Hessenberg column, V_{j+1} = W / ||W||.
static int batch_arnoldi_step(helm_batch_t b, int j, hipStream_t s) {
    const int ns = b->nsys, kk = b->restart, nt = b->ntiles, hstride = kk + 1;
    const SysVec* dsv = b->sv.as<SysVec>();
    const int32_t* dt = b->tiles.as<int32_t>();
    const int32_t* act = b->active.as<int32_t>();
    const MvDev none{nullptr, nullptr, nullptr, 0, 0};
    const int zprec = b->prec == HELM_C128 ? 0 : 1;
    int rc = batch_sweep(b, b->io_sweep.as<IoDev>() + (size_t)j * b->count, zprec, act, s);
    if (rc) return rc;
    {
        PhaseScope ph(PH_MATVEC, s);
        launch_matvec(b->probs.as<ProbDev>(), b->mv_z.as<MvDev>() + (size_t)j * b->count, none, b->mv_blk.as<int32_t>(),
                      b->count, b->mv_blocks, zprec, act, s);
        LAUNCHCHK();
    }
    PhaseScope phk(PH_KRYLOV, s, j + 1 <= KR_FUSE ? 9 : 10);
    double2* Hcol = b->H.as<double2>() + (size_t)j * (kk + 1);   // system stride kk*(kk+1)
    const int hs_ = kk * (kk + 1);
    launch_multidot(dsv, dt, ns, nt, j, b->partial.as<double2>(), hstride, act, s);
    launch_reduce_partials(dt, ns, b->partial.as<double2>(), hstride, j + 1, Hcol, hs_, 0, act, s);
    if (j + 1 <= KR_FUSE) {
        // first update and second dot products in one pass over V (same values as the two kernels)
        launch_multiaxpy_dot(dsv, dt, ns, nt, j, Hcol, hs_, b->partial.as<double2>(), hstride, act, s);
    } else {
        launch_multiaxpy(dsv, dt, ns, nt, j, Hcol, hs_, act, s);
        launch_multidot(dsv, dt, ns, nt, j, b->partial.as<double2>(), hstride, act, s);
    }
    launch_reduce_partials(dt, ns, b->partial.as<double2>(), hstride, j + 1, b->hbuf.as<double2>(), hstride, 0, act, s);
    launch_reduce_partials(dt, ns, b->partial.as<double2>(), hstride, j + 1, Hcol, hs_, 1, act, s);
    // second update, with the norm partials of the result (the dot partials are consumed above)
    launch_multiaxpy(dsv, dt, ns, nt, j, b->hbuf.as<double2>(), hstride, act, s, b->partial.as<double2>());
    launch_norm_finish(dt, ns, b->partial.as<double2>(), b->nrm.as<double>(), act, s);
    launch_arnoldi_finish(ns, j, kk, b->H.as<double2>(), b->cs.as<double2>(), b->g.as<double2>(), b->nrm.as<double>(),
                          b->inv.as<double>(), b->est.as<double>(), act, s);
    launch_scale_to_v(dsv, dt, ns, nt, j + 1, b->inv.as<double>(), act, s);
    LAUNCHCHK();
    return HELM_OK;
}

// x += Z y with y the least-squares solution of the cnt[s] Arnoldi steps of each system.
static int batch_update(helm_batch_t b, hipStream_t s) {
    const int zprec = b->prec == HELM_C128 ? 0 : 1;
    launch_backsolve(b->nsys, b->restart, b->H.as<double2>(), b->g.as<double2>(), b->cnt.as<int32_t>(),
                     b->y.as<double2>(), s);
    launch_update_x(b->sv.as<SysVec>(), b->tiles.as<int32_t>(), b->nsys, b->ntiles, b->cnt.as<int32_t>(),
                    b->y.as<double2>(), b->restart, zprec, s);
    LAUNCHCHK();
    return HELM_OK;
}

// Arnoldi steps per captured graph: after each chunk the host reads the flags once, so a cycle in which
// every system has converged stops within this many masked steps instead of running to the restart
// length, at restart / kGraphChunk host round trips per cycle instead of one per step.
constexpr int kGraphChunk = 4;

// The pieces of the graph form of one restart cycle, for systems flagged active; a system that
// converges leaves through its flag and its kernels then return at once.  Piece c < chunks: Arnoldi
// steps [c * kGraphChunk, ...) (the first also starts the cycle); piece `chunks`: the update, the new
// residual and the flags of the next cycle.  They read only batch-owned device memory, so one capture
// serves every later call on the batch.
static int batch_cycle_piece(helm_batch_t b, int piece, hipStream_t s) {
    const int ns = b->nsys, kk = b->restart;
    const int chunks = (kk + kGraphChunk - 1) / kGraphChunk;
    const CycleCtl* ctl = b->ctl.as<CycleCtl>();
    int rc;
    if (piece < chunks) {
        if (piece == 0) {
            launch_start_cycle(ns, b->beta.as<double>(), b->inv.as<double>(), b->g.as<double2>(), kk + 1, s);
            launch_scale_to_v(b->sv.as<SysVec>(), b->tiles.as<int32_t>(), ns, b->ntiles, 0, b->inv.as<double>(),
                              b->active.as<int32_t>(), s);
            LAUNCHCHK();
        }
        for (int j = piece * kGraphChunk; j < std::min(kk, (piece + 1) * kGraphChunk); ++j) {
            if ((rc = batch_arnoldi_step(b, j, s))) return rc;
            launch_iter_flags(ns, j, b->est.as<double>(), b->fnorm.as<double>(), ctl, b->it_d.as<int32_t>(),
                              b->cnt.as<int32_t>(), b->active.as<int32_t>(), s);
            LAUNCHCHK();
        }
        return HELM_OK;
    }
    if ((rc = batch_update(b, s))) return rc;
    if ((rc = batch_residual(b, s))) return rc;
    launch_cycle_flags(ns, b->beta.as<double>(), b->fnorm.as<double>(), ctl, b->it_d.as<int32_t>(), b->rr_d.as<double>(),
                       b->done_d.as<int32_t>(), b->active.as<int32_t>(), b->cnt.as<int32_t>(), s);
    LAUNCHCHK();
    return HELM_OK;
}

// Record every piece into a graph on the batch's own stream (a legacy null stream cannot capture)
// and instantiate it.  No timing events are recorded while capturing.
static int capture_cycle(helm_batch_t b) {
    if (!b->gstream) HIPCHK(hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking));
    const int pieces = (b->restart + kGraphChunk - 1) / kGraphChunk + 1;
    for (int c = 0; c < pieces; ++c) {
        HIPCHK(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
        timing().capturing = true;
        const int rc = batch_cycle_piece(b, c, b->gstream);
        timing().capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->gstream, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            b->drop_graph();
            return rc ? rc : fail(HELM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        }
        hipGraphExec_t x = nullptr;
        const hipError_t ei = hipGraphInstantiateWithFlags(&x, g, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->drop_graph();
            return fail(HELM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        b->gexec.push_back(x);
    }
    return HELM_OK;
}

extern "C" int helm_batch_set_graph(helm_batch_t b, int32_t on) {
    if (!b) return fail(HELM_EINVAL, "NULL argument");
    b->use_graph = on != 0;
    if (!b->use_graph) b->drop_graph();
    return HELM_OK;
}

extern "C" int fgmres_solve_batch(helm_batch_t b, const void* const* f, void* const* u, double tol, int32_t maxit,
                                  int32_t* iters, double* relres, void* stream) {
    if (!b || !f || !u) return fail(HELM_EINVAL, "NULL argument");
    if (!(tol > 0.0 && tol < 1.0)) return fail(HELM_EINVAL, "tol must be in (0, 1)");
    if (maxit < 1) return fail(HELM_EINVAL, "maxit must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const int ns = b->nsys, kk = b->restart, nt = b->ntiles;
    // per-call vector tables
    std::vector<SysVec> sv(ns);
    std::vector<MvDev> mvr(b->count);
    for (int p = 0, s0 = 0; p < b->count; s0 += b->nrhs[p], ++p) {
        if (!f[p] || !u[p]) return fail(HELM_EINVAL, "NULL vector for problem %d", p);
        mvr[p] = MvDev{u[p], b->W.as<double2>() + b->woff[p], f[p], b->nrhs[p], s0};
    }
    for (int sidx = 0; sidx < ns; ++sidx) {
        const int p = b->sys_prob[sidx], q = b->sys_rhs[sidx];
        const int64_t Np = b->N[p], R = b->nrhs[p];
        SysVec& v = sv[sidx];
        v.v = b->V.as<double2>() + b->voff[p] + q * Np;
        v.z = b->Z.as<char>() + b->zelem * (b->zoff[p] + q * Np);
        v.w = b->W.as<double2>() + b->woff[p] + q * Np;
        v.x = (double2*)u[p] + q * Np;
        v.f = (const double2*)f[p] + q * Np;
        v.len = Np;
        v.vstride = R * Np;
        v.zstride = R * Np;
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(b->sv.p, sv.data(), sizeof(SysVec) * ns, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->mv_res.p, mvr.data(), sizeof(MvDev) * b->count, hipMemcpyHostToDevice));
    const SysVec* dsv = b->sv.as<SysVec>();
    const int32_t* dt = b->tiles.as<int32_t>();

    std::vector<double> fn(ns), bet(ns), est(ns);
    std::vector<int32_t> it(ns, 0), done(ns, 0), act(ns, 0), cnt(ns, 0);
    std::vector<double> rr(ns, 0.0);
    launch_norms(dsv, dt, ns, nt, 1, b->partial.as<double2>(), b->fnorm.as<double>(), nullptr, s);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(fn.data(), b->fnorm.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < ns; ++i)
        if (!std::isfinite(fn[i])) return fail(HELM_EINVAL, "right-hand side %d has non-finite values", i);

    int rc;
    if (b->use_graph) {
        // Graph form: the host only replays whole cycles and reads the flags between them.
        const CycleCtl c{tol, maxit, 0};
        HIPCHK(hipMemcpy(b->ctl.p, &c, sizeof(c), hipMemcpyHostToDevice));
        launch_zero_i32(b->it_d.as<int32_t>(), ns, s);
        LAUNCHCHK();
        if ((rc = batch_residual(b, s))) return rc;
        launch_cycle_flags(ns, b->beta.as<double>(), b->fnorm.as<double>(), b->ctl.as<CycleCtl>(), b->it_d.as<int32_t>(),
                           b->rr_d.as<double>(), b->done_d.as<int32_t>(), b->active.as<int32_t>(), b->cnt.as<int32_t>(),
                           s);
        LAUNCHCHK();
        if (b->gexec.empty() && (rc = capture_cycle(b))) return rc;
        const int chunks = (int)b->gexec.size() - 1;
        auto any_active = [&]() -> int {
            if (hipMemcpyAsync(act.data(), b->active.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return -1;
            for (int i = 0; i < ns; ++i)
                if (act[i]) return 1;
            return 0;
        };
        while (true) {
            HIPCHK(hipMemcpyAsync(rr.data(), b->rr_d.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
            const int go = any_active();
            if (go < 0) return fail(HELM_EHIP, "reading the convergence flags");
            for (int i = 0; i < ns; ++i)
                if (!std::isfinite(rr[i])) return fail(HELM_EINVAL, "non-finite residual (system %d)", i);
            if (!go) break;
            for (int c = 0; c < chunks; ++c) {
                HIPCHK(hipGraphLaunch(b->gexec[c], s));
                if (c + 1 < chunks) {
                    const int more = any_active();
                    if (more < 0) return fail(HELM_EHIP, "reading the convergence flags");
                    if (!more) break;
                }
            }
            HIPCHK(hipGraphLaunch(b->gexec[chunks], s));
        }
        HIPCHK(hipMemcpyAsync(it.data(), b->it_d.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(done.data(), b->done_d.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        while (true) {
            if ((rc = batch_residual(b, s))) return rc;
            HIPCHK(hipMemcpyAsync(bet.data(), b->beta.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            int nact = 0;
            for (int i = 0; i < ns; ++i) {
                rr[i] = fn[i] > 0.0 ? bet[i] / fn[i] : 0.0;
                if (!std::isfinite(rr[i])) return fail(HELM_EINVAL, "non-finite residual (system %d)", i);
                done[i] = (rr[i] <= tol) || fn[i] == 0.0;
                act[i] = !done[i] && it[i] < maxit;
                cnt[i] = 0;
                nact += act[i];
            }
            if (nact == 0) break;
            HIPCHK(hipMemcpyAsync(b->active.p, act.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
            launch_start_cycle(ns, b->beta.as<double>(), b->inv.as<double>(), b->g.as<double2>(), kk + 1, s);
            LAUNCHCHK();
            launch_scale_to_v(dsv, dt, ns, nt, 0, b->inv.as<double>(), b->active.as<int32_t>(), s);
            LAUNCHCHK();
            for (int j = 0; j < kk; ++j) {
                if ((rc = batch_arnoldi_step(b, j, s))) return rc;
                HIPCHK(hipMemcpyAsync(est.data(), b->est.p, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                int still = 0;
                for (int i = 0; i < ns; ++i) {
                    if (!act[i]) continue;
                    it[i] += 1;
                    cnt[i] = j + 1;
                    const double e = est[i] / fn[i];
                    if (!(e > tol) || it[i] >= maxit) act[i] = 0;   // NaN estimate also ends the cycle
                    still += act[i];
                }
                if (still == 0 || j == kk - 1) break;
                HIPCHK(hipMemcpyAsync(b->active.p, act.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
            }
            HIPCHK(hipMemcpyAsync(b->cnt.p, cnt.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
            if ((rc = batch_update(b, s))) return rc;
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    bool all = true;
    for (int i = 0; i < ns; ++i) {
        if (iters) iters[i] = it[i];
        if (relres) relres[i] = rr[i];
        all = all && done[i];
    }
    return all ? HELM_OK : fail(HELM_ENOTCONV, "maxit reached before tol");
}

extern "C" int fgmres_solve(helm_problem_t A, sweep_factors_t M, const void* f, void* u, int32_t nrhs, int32_t restart,
                            double tol, int32_t maxit, int32_t* iters, double* relres, void* stream) {
    if (!A || !M || !f || !u) return fail(HELM_EINVAL, "NULL argument");
    if (M->A != A) return fail(HELM_EINVAL, "factors do not belong to this problem");
    if (nrhs < 1) return fail(HELM_EINVAL, "nrhs must be >= 1");
    if (!M->solo || M->solo_nrhs != nrhs || M->solo_restart != restart) {
        if (M->solo) { helm_batch_free(M->solo); M->solo = nullptr; }
        int rc = helm_batch_create(&A, &M, &nrhs, 1, restart, stream, &M->solo);
        if (rc) return rc;
        M->solo_nrhs = nrhs;
        M->solo_restart = restart;
    }
    return fgmres_solve_batch(M->solo, &f, &u, tol, maxit, iters, relres, stream);
}
