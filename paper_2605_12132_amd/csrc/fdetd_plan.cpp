// Host runtime of the FDETD library: plans, scratch ownership, the per-step launch sequence, hipGraph
// capture of the time loop, and the C-ABI declared in include/fdetd.h.
//
// One step of a Maxwell problem (section 2.1 midpoint solution, section 2.5 algorithm) is evaluated as a
// Horner recurrence with the source folded in:
//     psi' = sum_n (dt^n/n!) H^n (psi - dt 2^-n Jbar) = v_0,
//     v_N = w_N,  v_n = w_n + dt/(n+1) H v_{n+1},  w_n = psi - dt 2^-n Jbar,
// the same polynomial as T_N(dt H) psi - dt T_N(dt H/2) Jbar with N instead of 2N applications of H.
// The first stage forms w_N while loading psi, intermediate v_n ping-pong between two plan buffers and
// the last stage writes psi in place.  The envelope step is the same recurrence without source.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdetd.h"
#include "fdetd_internal.h"
#include "fdetd_tiles.h"

using namespace fdetd;

namespace {

thread_local std::string g_last_error;

struct Prob {
    fdetd_problem_desc d{};
    int nd = 0;
    size_t cells = 0;           // nz * nr
    void *buf[2] = {nullptr, nullptr};  // stage vectors (6 planes Maxwell, 2 planes envelope)
    void *jbar = nullptr;       // staggered J_rho plane
    float *lo = nullptr;        // FP32C compensation words (6 or 2 planes of float2)
    double *rinv_p = nullptr, *rinv_s = nullptr, *m2rinv2 = nullptr;
    double *sz = nullptr, *sr = nullptr;  // envelope absorbing layer: sigma per column and per row
    double *band = nullptr;               // current correction: LU factors of the radial operator
    double *gresp = nullptr;              // ... segment responses, forward then backward ([nr][nd] each)
    int seg = 0, nseg = 0;                // ... rows per segment of the partitioned solve, segments
    void *jth = nullptr;                  // current correction: corrected J_theta plane
    void *pbuf = nullptr;                 // FP32C increment form: P = H psi of the step (6 planes of float2)
    void *fine = nullptr;                 // 2x supersampled gather: 24 planes (4 position sets per component),
                                          // allocated on first use
    int lz = 0, lr = 0;                   // its widths (0, 0: no layer)
    double a[kMaxND], s[kMaxND], d1[kMaxND], d2[kMaxND + 1], c[kMaxND];
    const void *last_state = nullptr;   // psi (or a) of the previous call, for the FP32C reset rule
    double rho_hat = 0.0;
};

}  // namespace

// Problems of equal N_D, N and dt that share one launch per stage (FP32C: two, the near-axis segments
// separately): table entries [d0, d0 + count).
struct Batch {
    int nd, N, d0, count, ntiles, ntiles_ax;
    int seg;                   // rows per marching segment of the main launch
    int nt_store = 0;          // Maxwell stage outputs stored non-temporal (autotuned)
    int tile_order = 0;        // numbering of the Maxwell tiles (ProbDesc::tile_order, autotuned)
    int lane = 0;              // stream of the batch's launches: 0 = the plan's stream, l > 0 = lanes[l - 1]
    double dt;
    std::vector<int> members;  // user indices, in table order
};

struct fdetd_plan_s {
    int precision = FDETD_FP64;
    uint32_t flags = 0;
    int kind = FDETD_MAXWELL;
    hipStream_t stream = nullptr;
    std::vector<Prob> probs;
    std::vector<Batch> batches;
    std::vector<ProbDesc> desc;   // host copy of the device table
    ProbDesc *ddesc = nullptr;
    std::string err;
    fdetd_plan_info info{};
    // cached graph of the last captured call
    hipGraphExec_t gexec = nullptr;
    std::vector<const void *> gkey;
    // FDETD_PLAN_PROFILE: event pairs around stage kernels, pending until the next query
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<double> ev_bytes;
    bool adopt_next = false;  // fdetd_import_state: the next call keeps the imported words for its pointers
    std::vector<int> seg_rows;  // per launch batch: rows per marching segment of the main launch
    std::vector<int> nt_store;  // per launch batch: store policy of the Maxwell stage outputs
    std::vector<int> tile_order;  // per launch batch: tile numbering
    // side streams of a plan whose launch batches run concurrently, with the fork and join events
    std::vector<hipStream_t> lanes;
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    // FP32C batches that mix widths: the near-axis launch of each stage runs on this stream beside the
    // main launch, forked and joined around the stage
    hipStream_t axis_stream = nullptr;
    hipEvent_t axis_fork = nullptr, axis_join = nullptr;
    void *zero = nullptr;  // FP32C increment form: 6 zero planes of the largest problem
};

namespace {

int fail(fdetd_plan_t p, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (p)
        p->err = buf;
    else
        g_last_error = buf;
    return code;
}

#define HIPCHK(p, call)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail((p), e_ == hipErrorOutOfMemory ? FDETD_E_NOMEM : FDETD_E_HIP, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                          \
    } while (0)

size_t elem_bytes(int precision) { return precision == FDETD_FP64 ? 16 : 8; }
int prec_code(int precision) { return precision == FDETD_FP64 ? P64 : P32; }
int planes(int kind) { return kind == FDETD_MAXWELL ? 6 : 2; }

double parity_mS(int m) { return (m % 2 == 0) ? 1.0 : -1.0; }

// Rows next to the axis that FP32C plans compute in FP64 arithmetic: the 2 N_D rows whose stencils reach
// the axis ghosts and the largest 1/rho factors, or the count in FDETD_AXIS_ROWS (0 .. 4096; 0 = none), read
// when a plan is made (for measuring what the FP64 band buys).
int axis_band_rows(int nd)
{
    if (const char *e = std::getenv("FDETD_AXIS_ROWS")) {
        char *end = nullptr;
        const long v = std::strtol(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0 && v <= 4096) return (int)v;
    }
    return 2 * nd;
}

void free_prob(Prob &q)
{
    for (void *b : q.buf)
        if (b) (void)hipFree(b);
    if (q.jbar) (void)hipFree(q.jbar);
    if (q.lo) (void)hipFree(q.lo);
    if (q.rinv_p) (void)hipFree(q.rinv_p);
    if (q.rinv_s) (void)hipFree(q.rinv_s);
    if (q.m2rinv2) (void)hipFree(q.m2rinv2);
    if (q.sz) (void)hipFree(q.sz);
    if (q.band) (void)hipFree(q.band);
    if (q.gresp) (void)hipFree(q.gresp);
    if (q.jth) (void)hipFree(q.jth);
    if (q.sr) (void)hipFree(q.sr);
    if (q.fine) (void)hipFree(q.fine);
    if (q.pbuf) (void)hipFree(q.pbuf);
    q = Prob{};
}

void fill_maxwell_args(const fdetd_plan_t P, const Prob &q, MaxwellStageArgs &A)
{
    std::memset(&A, 0, sizeof A);
    A.rinv_p = q.rinv_p;
    A.rinv_s = q.rinv_s;
    A.dr = q.d.dr;
    A.pS = parity_mS(q.d.m);
    A.nz = q.d.nz;
    A.nr = q.d.nr;
    A.m = q.d.m;
    A.axis_rows = P->precision == FDETD_FP32C ? axis_band_rows(q.nd) : 0;
    for (int j = 0; j < q.nd; ++j) {
        A.az[j] = q.a[j] / q.d.dz;
        A.ar[j] = q.a[j] / q.d.dr;
        A.cax[j] = q.c[j];
    }
}

void fill_envelope_args(const fdetd_plan_t P, const Prob &q, EnvelopeStageArgs &A)
{
    std::memset(&A, 0, sizeof A);
    A.rinv_p = q.rinv_p;
    A.m2rinv2 = q.m2rinv2;
    A.k0 = q.d.k0;
    A.pS = parity_mS(q.d.m);
    A.nz = q.d.nz;
    A.nr = q.d.nr;
    A.axis_rows = P->precision == FDETD_FP32C ? axis_band_rows(q.nd) : 0;
    for (int j = 0; j <= q.nd; ++j) {
        A.bz[j] = q.d2[j] / (q.d.dz * q.d.dz);
        A.br[j] = q.d2[j] / (q.d.dr * q.d.dr);
    }
    for (int j = 0; j < q.nd; ++j) {
        A.dzc[j] = q.d1[j] / q.d.dz;
        A.drc[j] = q.d1[j] / q.d.dr;
    }
}

// FDETD_PLAN_PROFILE: record an event pair around the next stage kernel.
int profile_begin(fdetd_plan_t P, double bytes)
{
    if (!(P->flags & FDETD_PLAN_PROFILE)) return FDETD_OK;
    while (P->ev_pool.size() < P->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(P, hipEventCreate(&e));
        P->ev_pool.push_back(e);
    }
    HIPCHK(P, hipEventRecord(P->ev_pool[P->ev_used], P->stream));
    P->ev_bytes.push_back(bytes);
    return FDETD_OK;
}

int profile_end(fdetd_plan_t P)
{
    if (!(P->flags & FDETD_PLAN_PROFILE)) return FDETD_OK;
    HIPCHK(P, hipEventRecord(P->ev_pool[P->ev_used + 1], P->stream));
    P->ev_used += 2;
    return FDETD_OK;
}

// Zero fill of plan-owned words.  Called from fdetd_step / envelope_step before any graph capture, so
// it never becomes a node of a captured graph.
int zero_device(fdetd_plan_t P, void *ptr, size_t bytes)
{
    HIPCHK(P, hipMemsetAsync(ptr, 0, bytes, P->stream));
    return FDETD_OK;
}

// One stage of one launch batch: the main tiles and, FP32C, the near-axis tiles in one launch.
int launch_stage(fdetd_plan_t P, const Batch &b, BatchArgs &A, hipStream_t s)
{
    const int prec = prec_code(P->precision);
    A.ntiles = b.ntiles;
    A.ntiles_ax = b.ntiles_ax;
    if (A.ntiles + A.ntiles_ax == 0) return FDETD_OK;
    if (P->kind == FDETD_MAXWELL && b.nd < 0 && P->axis_stream && A.ntiles && A.ntiles_ax) {
        // widths mixed in FP32 storage: the near-axis tiles (FP64 arithmetic, a launch of their own) run on
        // the axis stream beside the main tiles.  Both read only vectors that the stage does not write
        // (the previous stage's, psi, Jbar) away from their own rows, and write disjoint rows.
        BatchArgs X = A, M = A;
        X.ntiles = 0;
        M.ntiles_ax = 0;
        HIPCHK(P, hipEventRecord(P->axis_fork, s));
        HIPCHK(P, hipStreamWaitEvent(P->axis_stream, P->axis_fork, 0));
        HIPCHK(P, launch_maxwell_any(prec, X, P->axis_stream));
        HIPCHK(P, launch_maxwell_any(prec, M, s));
        HIPCHK(P, hipEventRecord(P->axis_join, P->axis_stream));
        HIPCHK(P, hipStreamWaitEvent(s, P->axis_join, 0));
        return FDETD_OK;
    }
    if (P->kind == FDETD_MAXWELL)
        HIPCHK(P, b.nd > 0 ? launch_maxwell_march(prec, b.nd, A, s) : launch_maxwell_any(prec, A, s));
    else
        HIPCHK(P, launch_envelope_march(prec, b.nd, A, s));
    return FDETD_OK;
}

// Whether the first Horner stage of batch b forms the E part of w_N itself (as it loads psi and Jbar)
// instead of reading it from a plane that a separate pass wrote: the Horner form, except FP32C at N = 1,
// where the first stage is also the compensated last one.
bool fuse_wn(const fdetd_plan_t P, const Batch &b, bool has_current)
{
    return has_current && !(P->flags & FDETD_PLAN_INCREMENT_FORM) &&
           !(P->precision == FDETD_FP32C && b.N == 1) && !(P->flags & FDETD_PLAN_SEPARATE_WN);
}

// One Maxwell step of the problems of batch b on stream s: stage the currents, N Horner stages, then the
// N = 1 copy and, at the end of a call, the axis rule of each problem.
int enqueue_maxwell_batch(fdetd_plan_t P, const Batch &b, void *const *psi, const void *const *j,
                          int last_step_of_call, hipStream_t s)
{
    const int prec = prec_code(P->precision);
    const size_t eb = elem_bytes(P->precision);
    BatchArgs A;
    std::memset(&A, 0, sizeof A);
    A.probs = P->ddesc + b.d0;
    A.nprob = b.count;
    A.ntiles = b.ntiles;
    A.ntiles_ax = b.ntiles_ax;
    size_t cells = 0;
    for (int t = 0; t < b.count; ++t) {
        A.psi[t] = psi[b.members[t]];
        A.aux[t] = j ? j[b.members[t]] : nullptr;
        cells += P->probs[b.members[t]].cells;
    }
    if (j && b.ntiles + b.ntiles_ax)
        HIPCHK(P, b.nd > 0 ? launch_stagger_march(prec, b.nd, A, s) : launch_stagger_any(prec, A, s));
    if (j && (P->flags & FDETD_PLAN_CURRENT_CORRECTION)) {
        // divergence error per problem, the banded solves of up to kMaxSolve problems per launch, then the
        // corrected currents per problem
        std::vector<CorrectArgs> X(b.count);
        SolveArgs S;
        std::memset(&S, 0, sizeof S);
        S.nd = b.nd;
        for (int t = 0; t < b.count; ++t) {
            const int p = b.members[t];
            const Prob &q = P->probs[p];
            const size_t pb = q.cells * eb;
            CorrectArgs &x = X[t];
            std::memset(&x, 0, sizeof x);
            x.jbar = q.jbar;
            x.jth_in = (const char *)j[p] + pb;
            x.rho_xy = (const char *)j[p] + 3 * pb;
            x.jth_out = q.jth;
            x.work = (double2 *)q.buf[1];  // free until the second stage; holds >= 16 B per cell
            x.band = q.band;
            x.nz = q.d.nz;
            x.nr = q.d.nr;
            x.nd = q.nd;
            x.m = q.d.m;
            x.parity = parity_mS(q.d.m);
            x.dr = q.d.dr;
            for (int u = 0; u < q.nd; ++u) x.a[u] = q.a[u];
            HIPCHK(P, launch_correct_div(prec, x, s));
            // boundary values of the partitioned solve after the work plane in the same buffer: at most
            // nseg * nd <= 2 nr rows of 16 B, within the 6 planes of 8 or 16 B it holds
            S.p[S.nprob] = {x.work, x.work + q.cells, q.band, q.gresp, q.gresp + (size_t)q.d.nr * q.nd, q.d.nz,
                            q.d.nr, q.seg, q.nseg};
            S.smax = std::max(S.smax, q.nseg);
            if (++S.nprob == kMaxSolve || t == b.count - 1) {
                HIPCHK(P, launch_correct_solve(S, s));
                S.nprob = 0;
                S.smax = 0;
            }
        }
        for (int t = 0; t < b.count; ++t) HIPCHK(P, launch_correct_apply(prec, X[t], s));
    }
    A.N = b.N;
    A.has_src = j != nullptr;
    A.compensated = P->precision == FDETD_FP32C;
    A.increment = (P->flags & FDETD_PLAN_INCREMENT_FORM) ? 1 : 0;
    A.fuse_wn = fuse_wn(P, b, j != nullptr);
    A.nt_store = b.nt_store;
    if (A.increment && b.ntiles + b.ntiles_ax) {
        // P = H psi of the step in two passes, H lo from zero, then P += H psi_hi (coef 1, no current), with
        // the stages' own operator (float stencils, FP64 near-axis rows): an operator for P that differed
        // from the stages' by the rounding of its coefficients would put that difference into the step's
        // dt^2 term, a steady drift of the energy instead of rounding noise
        A.has_src = 0;
        A.n = b.N - 1;
        A.beta_in = A.beta = 0.0;
        A.coef = 1.0;
        for (int role = 1; role <= 2; ++role) {
            A.role = role;
            int rc = profile_begin(P, 18.0 * cells * eb);
            if (rc) return rc;
            if ((rc = launch_stage(P, b, A, s))) return rc;
            if ((rc = profile_end(P))) return rc;
        }
        A.role = 0;
        A.has_src = j != nullptr;
    }
    if (j && b.ntiles + b.ntiles_ax && !A.fuse_wn) {
        // E part of w_N = psi + beta_in Jbar into buf[1] (increment form: of d_N = beta_in Jbar): read by the
        // B half of the first stage
        A.beta_in = -b.dt * std::ldexp(1.0, -b.N);
        size_t max_cells = 0;
        for (int t = 0; t < b.count; ++t) max_cells = std::max(max_cells, P->probs[b.members[t]].cells);
        HIPCHK(P, launch_form_wn(prec, A, max_cells, s));
    }
    for (int n = b.N - 1; n >= 0; --n) {
        A.n = n;
        A.beta_in = -b.dt * std::ldexp(1.0, -b.N);
        A.beta = -b.dt * std::ldexp(1.0, -n);
        A.coef = b.dt / (n + 1);
        // algorithmic bytes: vin (6c) + psi (6c) + Jbar (3c) + vout (6c); the first stage without a current
        // reads psi once as vin and as psi (12c); with one, its B half reads w_N from buf[1], or, fused,
        // psi's E part and Jbar again (3c more)
        const double cvals = (n == b.N - 1 && !j ? 12.0 : 18.0) + (j ? 3.0 : 0.0) + (n == b.N - 1 && A.fuse_wn ? 3.0 : 0.0);
        const double bytes = cvals * cells * eb + (A.compensated && n == 0 ? 2.0 * 6 * cells * 8 : 0.0) +
                             (A.increment && n == 0 ? 6.0 * cells * eb : 0.0);
        int rc = profile_begin(P, bytes);
        if (rc) return rc;
        if ((rc = launch_stage(P, b, A, s))) return rc;
        if ((rc = profile_end(P))) return rc;
    }
    int max_nz = 0;
    for (int t = 0; t < b.count; ++t) {
        const int p = b.members[t];
        const Prob &q = P->probs[p];
        if (q.d.taylor_order == 1 && !A.increment) HIPCHK(P, launch_copy(q.buf[0], psi[p], 6 * q.cells * eb, s));
        max_nz = std::max(max_nz, q.d.nz);
    }
    if (last_step_of_call) HIPCHK(P, launch_axis_fix_batch(prec, A, max_nz, s));
    return FDETD_OK;
}

// exp(-sigma dt/4) on the absorbing layers of the problems of batch b that have one.
int damp_layers(fdetd_plan_t P, const Batch &b, void *const *a, void *const *at, hipStream_t s)
{
    for (int t = 0; t < b.count; ++t) {
        const int p = b.members[t];
        const Prob &q = P->probs[p];
        if (q.lz == 0 && q.lr == 0) continue;
        DampArgs X{};
        X.a = a[p];
        X.at = at[p];
        X.lo = q.lo;
        X.sz = q.sz;
        X.sr = q.sr;
        X.nz = q.d.nz;
        X.nr = q.d.nr;
        X.lz = q.lz;
        X.lr = q.lr;
        X.qdt = q.d.dt / 4.0;
        HIPCHK(P, launch_absorb_damp(prec_code(P->precision), X, s));
    }
    return FDETD_OK;
}

// One envelope step of the problems of batch b on stream s.
int enqueue_envelope_batch(fdetd_plan_t P, const Batch &b, void *const *a, void *const *at, const void *const *chi,
                           hipStream_t s)
{
    const size_t eb = elem_bytes(P->precision);
    BatchArgs A;
    std::memset(&A, 0, sizeof A);
    A.probs = P->ddesc + b.d0;
    A.nprob = b.count;
    A.ntiles = b.ntiles;
    A.N = b.N;
    A.compensated = P->precision == FDETD_FP32C;
    size_t cells = 0;
    for (int t = 0; t < b.count; ++t) {
        A.psi[t] = a[b.members[t]];
        A.aux[t] = at[b.members[t]];
        A.chi[t] = chi[b.members[t]];
        cells += P->probs[b.members[t]].cells;
    }
    int rc = damp_layers(P, b, a, at, s);  // first factor exp(-sigma dt/4) of the split step
    if (rc) return rc;
    A.increment = (P->flags & FDETD_PLAN_INCREMENT_FORM) ? 1 : 0;
    if (A.increment && b.ntiles + b.ntiles_ax) {
        // P = H_a psi of the step (of the damped state), H_a lo from zero, then P += H_a psi_hi, with the
        // stages' own operator; chi of the step in both
        A.n = b.N - 1;
        A.coef = 1.0;
        for (int role = 1; role <= 2; ++role) {
            A.role = role;
            if ((rc = profile_begin(P, 6.5 * cells * eb))) return rc;
            if ((rc = launch_stage(P, b, A, s))) return rc;
            if ((rc = profile_end(P))) return rc;
        }
        A.role = 0;
    }
    for (int n = b.N - 1; n >= 0; --n) {
        A.n = n;
        A.coef = b.dt / (n + 1);
        // algorithmic bytes: vin (2c) + psi (2c; the same data in the first stage) + chi + vout (2c)
        const double cvals = (n == b.N - 1 ? 4.0 : 6.0) + 0.5;
        const double bytes = cvals * cells * eb + (A.compensated && n == 0 ? 2.0 * 2 * cells * 8 : 0.0);
        if ((rc = profile_begin(P, bytes))) return rc;
        if ((rc = launch_stage(P, b, A, s))) return rc;
        if ((rc = profile_end(P))) return rc;
    }
    for (int t = 0; t < b.count; ++t) {
        const int p = b.members[t];
        const Prob &q = P->probs[p];
        if (q.d.taylor_order == 1 && !A.increment) {
            const size_t plane_b = q.cells * eb;
            HIPCHK(P, launch_copy(q.buf[0], a[p], plane_b, s));
            HIPCHK(P, launch_copy((char *)q.buf[0] + plane_b, at[p], plane_b, s));
        }
    }
    return damp_layers(P, b, a, at, s);  // second factor
}

// Planes of one current block: J_rho, J_theta, J_z, and with the current correction rho_xy.
int cur_planes(const fdetd_plan_t P) { return (P->flags & FDETD_PLAN_CURRENT_CORRECTION) ? 4 : 3; }

// LU factors (no pivoting) of the radial operator L_rho^(mS) - m^2/rho^2 of section 3.7 on nr primary
// rows, as rows of 2 nd + 1: L(k, k - j) at nd - j, 1 / U(k, k) at nd, U(k, k + j) at nd + j.
// L_rho phi(k) = (b_0 phi_k + sum_j b_j (phi_(k+j) + phi_(k-j))) / dr^2 + sum_j d_j (phi_(k+j) - phi_(k-j)) / (rho_k dr),
// rows below the axis mirrored with the m_S sign, rows from nr on 0.  False on a vanishing pivot.
bool radial_lu(const Prob &q, std::vector<double> &band)
{
    const int nd = q.nd, nr = q.d.nr, W = 2 * nd + 1, m = q.d.m;
    const double dr = q.d.dr, ps = parity_mS(m);
    band.assign((size_t)nr * W, 0.0);
    auto at = [&](int k, int c) -> double & { return band[(size_t)k * W + nd + (c - k)]; };
    for (int k = 0; k < nr; ++k) {
        const double rho = (k + 0.5) * dr;
        at(k, k) += q.d2[0] / (dr * dr) - (double)m * m / (rho * rho);
        for (int j = 1; j <= nd; ++j) {
            const double cp = q.d2[j] / (dr * dr) + q.d1[j - 1] / (rho * dr);
            const double cm = q.d2[j] / (dr * dr) - q.d1[j - 1] / (rho * dr);
            if (k + j < nr) at(k, k + j) += cp;
            const int r = k - j;
            if (r >= 0) at(k, r) += cm;
            else if (-1 - r < nr) at(k, -1 - r) += ps * cm;
        }
    }
    for (int k = 0; k < nr; ++k) {
        const double piv = at(k, k);
        if (!(std::fabs(piv) > 1e-300) || !std::isfinite(piv)) return false;
        const int last = std::min(k + nd, nr - 1);
        for (int i = k + 1; i <= last; ++i) {
            const double l = at(i, k) / piv;
            at(i, k) = l;
            for (int c = k + 1; c <= last; ++c) at(i, c) -= l * at(k, c);
        }
    }
    for (int k = 0; k < nr; ++k) at(k, k) = 1.0 / at(k, k);
    return true;
}

// Responses of the partitioned solve (rows split into nseg segments of seg rows): for each segment but the
// first of a pass, the values its rows take from a zero right-hand side when boundary value t is 1 and the
// others 0.  Forward boundary t = y(a - 1 - t), backward x(b + t), for a segment [a, b).  Out: gresp =
// forward [nr][nd] then backward [nr][nd].
void segment_responses(const Prob &q, const std::vector<double> &band, int seg, std::vector<double> &gresp)
{
    const int nd = q.nd, nr = q.d.nr, W = 2 * nd + 1, ns = (nr + seg - 1) / seg;
    gresp.assign((size_t)2 * nr * nd, 0.0);
    double *gf = gresp.data(), *gb = gresp.data() + (size_t)nr * nd;
    std::vector<double> v(nr);
    for (int s = 0; s < ns; ++s) {
        const int a = s * seg, b = std::min(nr, a + seg);
        for (int t0 = 0; t0 < nd; ++t0) {
            if (s >= 1) {  // forward
                std::fill(v.begin(), v.end(), 0.0);
                for (int t = 0; t < nd; ++t)
                    if (a - 1 - t >= 0) v[a - 1 - t] = t == t0 ? 1.0 : 0.0;
                for (int k = a; k < b; ++k) {
                    double y = 0.0;
                    for (int j = 1; j <= nd && k - j >= 0; ++j) y -= band[(size_t)k * W + nd - j] * v[k - j];
                    v[k] = y;
                    gf[(size_t)k * nd + t0] = y;
                }
            }
            if (s <= ns - 2) {  // backward
                std::fill(v.begin(), v.end(), 0.0);
                for (int t = 0; t < nd; ++t)
                    if (b + t < nr) v[b + t] = t == t0 ? 1.0 : 0.0;
                for (int k = b - 1; k >= a; --k) {
                    double x = 0.0;
                    for (int j = 1; j <= nd && k + j < nr; ++j) x -= band[(size_t)k * W + nd + j] * v[k + j];
                    x *= band[(size_t)k * W + nd];
                    v[k] = x;
                    gb[(size_t)k * nd + t0] = x;
                }
            }
        }
    }
}

// Launch batches hold disjoint problems, so a call can run them on several streams: the side streams
// wait for an event recorded on the plan's stream when the call starts, and the plan's stream waits for
// an event recorded on each side stream when it ends.  Under graph capture the same pattern gives a
// graph with one branch per stream.
int fork_lanes(fdetd_plan_t P)
{
    if (P->lanes.empty()) return FDETD_OK;
    HIPCHK(P, hipEventRecord(P->fork_ev, P->stream));
    for (hipStream_t s : P->lanes) HIPCHK(P, hipStreamWaitEvent(s, P->fork_ev, 0));
    return FDETD_OK;
}

int join_lanes(fdetd_plan_t P)
{
    for (size_t l = 0; l < P->lanes.size(); ++l) {
        HIPCHK(P, hipEventRecord(P->join_ev[l], P->lanes[l]));
        HIPCHK(P, hipStreamWaitEvent(P->stream, P->join_ev[l], 0));
    }
    return FDETD_OK;
}

hipStream_t lane_stream(fdetd_plan_t P, const Batch &b) { return b.lane ? P->lanes[b.lane - 1] : P->stream; }

// Launch batches that mix stencil widths: Maxwell plans in FP64 or with FDETD_PLAN_MIXED_WIDTHS, unless
// FDETD_PLAN_PER_WIDTH, and never with the current correction, whose banded solves are batched per width.
// FP32C plans batch per width by default: their mixed launches split main and near-axis tiles into two
// launches per stage (the near-axis one on a stream of its own beside the main one), and per-width batches
// on four streams still measured ~3 % faster on the 64-problem batch.
bool mixed_widths(const fdetd_plan_t P)
{
    if (P->kind != FDETD_MAXWELL ||
        (P->flags & (FDETD_PLAN_CURRENT_CORRECTION | FDETD_PLAN_PER_WIDTH | FDETD_PLAN_INCREMENT_FORM)))
        return false;
    return (P->flags & FDETD_PLAN_MIXED_WIDTHS) || P->precision == FDETD_FP64;
}

// Streams of a plan with more than one launch batch: longest-processing-time assignment of the batches
// (work ~ cells x (N + 1)) to at most kMaxLanes streams, the plan's own stream being lane 0.  Profiled
// plans and FDETD_PLAN_ONE_STREAM keep every launch on the plan's stream.
// The stream of the near-axis launches of FP32C batches that mix widths (not when profiling or on one
// stream: then they follow the main launch on the batch's stream).
int make_axis_stream(fdetd_plan_t P)
{
    if (P->flags & (FDETD_PLAN_PROFILE | FDETD_PLAN_ONE_STREAM)) return FDETD_OK;
    bool need = false;
    for (const Batch &b : P->batches) need = need || (b.nd < 0 && b.ntiles && b.ntiles_ax);
    if (!need) return FDETD_OK;
    HIPCHK(P, hipStreamCreateWithFlags(&P->axis_stream, hipStreamNonBlocking));
    HIPCHK(P, hipEventCreateWithFlags(&P->axis_fork, hipEventDisableTiming));
    HIPCHK(P, hipEventCreateWithFlags(&P->axis_join, hipEventDisableTiming));
    return FDETD_OK;
}

int assign_lanes(fdetd_plan_t P)
{
    constexpr int kMaxLanes = 4;
    for (Batch &b : P->batches) b.lane = 0;
    const int nl = std::min<int>(kMaxLanes, (int)P->batches.size());
    if (nl < 2 || (P->flags & (FDETD_PLAN_PROFILE | FDETD_PLAN_ONE_STREAM))) return FDETD_OK;
    std::vector<int> order(P->batches.size());
    std::vector<double> work(P->batches.size(), 0.0), load(nl, 0.0);
    for (size_t i = 0; i < order.size(); ++i) {
        order[i] = (int)i;
        for (int p : P->batches[i].members) work[i] += (double)P->probs[p].cells * (P->batches[i].N + 1);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        P->batches[i].lane = l;
        load[l] += work[i];
    }
    HIPCHK(P, hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
    for (int l = 1; l < nl; ++l) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        HIPCHK(P, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        P->lanes.push_back(s);
        HIPCHK(P, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        P->join_ev.push_back(e);
    }
    return FDETD_OK;
}

// Rows per marching segment: long segments load each rho-stencilled row once per segment (the window
// warm-up costs 2 N_D - 1 extra rows), short ones give more wavefronts.  Default before autotuning: the
// longest segment (8 .. 64 rows) that still gives every SIMD of the chip (1024) one wavefront.
// Whether a batch's stage kernels exist with non-temporal output stores: per-width Maxwell launches of the
// Horner form (launches that mix widths and the increment form keep the default stores).
bool store_policy_applies(const fdetd_plan_t P, const Batch &b)
{
    return P->kind == FDETD_MAXWELL && b.nd > 0 && !(P->flags & FDETD_PLAN_INCREMENT_FORM);
}

// FDETD_STORE_POLICY = 0 or 1 fixes the store policy of the Maxwell stage outputs (no timing); -1: unset.
int forced_store_policy()
{
    if (const char *e = std::getenv("FDETD_STORE_POLICY")) {
        if (e[0] == '0' && e[1] == 0) return 0;
        if (e[0] == '1' && e[1] == 0) return 1;
    }
    return -1;
}

// FDETD_TILE_ORDER = 0 or 1 fixes the numbering of the Maxwell tiles (no timing); -1: unset.
int forced_tile_order()
{
    if (const char *e = std::getenv("FDETD_TILE_ORDER")) {
        if (e[0] == '0' && e[1] == 0) return 0;
        if (e[0] == '1' && e[1] == 0) return 1;
    }
    return -1;
}

int forced_seg_rows()
{
    if (const char *e = std::getenv("FDETD_SEG_ROWS")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 4096) return v;
    }
    return 0;
}
int default_seg_rows(int64_t row_strips_total)
{
    if (const int f = forced_seg_rows()) return f;
    int s = 8;
    while (s < 64 && row_strips_total / (2 * s) >= 1024) s *= 2;
    return s;
}
constexpr int kSegAxis = 16;  // rows per segment of the FP32C near-axis tiles (16: 1-2 % faster than 8 on
                               // the 64-problem batch and the LWFA-scale grid; 32 alike)
// FDETD_SEG_AXIS overrides it (1 .. 64 rows)
int axis_segment_rows()
{
    if (const char *e = std::getenv("FDETD_SEG_AXIS")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 64) return v;
    }
    return kSegAxis;
}

// Group problems into launch batches, fill the descriptor table and upload it.  P->seg_rows gives the
// segment length of each batch; when it does not match the batch count the defaults are taken.
int build_batches(fdetd_plan_t P)
{
    P->batches.clear();
    P->desc.clear();
    const bool have_segs = !P->seg_rows.empty();
    const int n = (int)P->probs.size();
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    // FDETD_PLAN_MIXED_WIDTHS: a batch holds problems of any stencil width (sorted by width inside it, so
    // that each XCD's contiguous tile range mostly runs one width's code); otherwise one width per batch
    const bool mixed = mixed_widths(P);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const auto &a = P->probs[x].d, &b = P->probs[y].d;
        if (!mixed && a.fd_order != b.fd_order) return a.fd_order < b.fd_order;
        if (a.taylor_order != b.taylor_order) return a.taylor_order < b.taylor_order;
        if (a.dt != b.dt) return a.dt < b.dt;
        return a.fd_order < b.fd_order;
    });
    const int halves = P->kind == FDETD_MAXWELL ? 2 : 1;
    const int cpw = march_columns_per_wave(prec_code(P->precision));
    for (int t = 0; t < n;) {
        const auto &d0 = P->probs[order[t]].d;
        Batch b;
        b.nd = d0.fd_order / 2;
        b.N = d0.taylor_order;
        b.dt = d0.dt;
        b.d0 = (int)P->desc.size();
        int64_t row_strips = 0;
        int u = t;
        while (u < n && u - t < kMaxBatch) {
            const auto &du = P->probs[order[u]].d;
            if ((!mixed && du.fd_order != d0.fd_order) || du.taylor_order != d0.taylor_order || du.dt != d0.dt) break;
            row_strips += (int64_t)halves * ((du.nz + cpw - 1) / cpw) * du.nr;
            ++u;
        }
        const size_t bi = P->batches.size();
        const int seg = have_segs && bi < P->seg_rows.size() ? P->seg_rows[bi] : default_seg_rows(row_strips);
        b.nt_store = bi < P->nt_store.size() ? P->nt_store[bi] : std::max(0, forced_store_policy());
        b.tile_order = bi < P->tile_order.size() ? P->tile_order[bi] : std::max(0, forced_tile_order());
        int tiles = 0, tiles_ax = 0;
        for (int v = t; v < u; ++v) {
            const Prob &q = P->probs[order[v]];
            ProbDesc D;
            describe_problem(q.d, P->precision, seg, D);
            D.tile_begin = tiles;
            D.tile_begin_ax = tiles_ax;
            D.tile_order = P->kind == FDETD_MAXWELL ? b.tile_order : 0;
            D.buf[0] = q.buf[0];
            D.buf[1] = q.buf[1];
            D.jbar = q.jbar;
            D.lo = q.lo;
            D.pbuf = q.pbuf;
            D.zero = P->zero;
            D.rinv_p = q.rinv_p;
            D.rinv_s = q.rinv_s;
            D.m2rinv2 = q.m2rinv2;
            D.sz = q.sz;
            D.jth = q.jth;
            D.sr = q.sr;
            tiles += halves * D.nseg * D.nstrip;
            tiles_ax += halves * D.nseg_ax * D.nstrip_ax;
            P->desc.push_back(D);
            b.members.push_back(order[v]);
        }
        b.count = u - t;
        for (int v = t; v < u; ++v)
            if (P->probs[order[v]].nd != b.nd) b.nd = -1;  // several widths: the launches that mix them
        b.seg = seg;
        b.ntiles = tiles;
        b.ntiles_ax = tiles_ax;
        if (!store_policy_applies(P, b)) b.nt_store = 0;
        P->batches.push_back(b);
        t = u;
    }
    // the near-axis and main tiles together must produce every (half, z column, rho row) of each problem
    // exactly once, from tiles that stay inside the grid (columns counted in units of kAxisColumns, which
    // divides the main tiles' width)
    if (cpw % kAxisColumns) return fail(P, FDETD_E_ARG, "internal: tile widths");
    for (const Batch &b : P->batches)
        for (int t = 0; t < b.count; ++t) {
            const ProbDesc &D = P->desc[b.d0 + t];
            const int units = (D.nz + kAxisColumns - 1) / kAxisColumns;
            std::vector<unsigned char> seen((size_t)halves * units * D.nr, 0);
            for (int axis = 0; axis < 2; ++axis) {
                const int w = axis ? axis_columns(D.nd) : cpw;
                const int nl = halves * (axis ? D.nseg_ax * D.nstrip_ax : D.nseg * D.nstrip);
                int begin = 0;
                for (int u = 0; u < t; ++u) {
                    const ProbDesc &E = P->desc[b.d0 + u];
                    begin += halves * (axis ? E.nseg_ax * E.nstrip_ax : E.nseg * E.nstrip);
                }
                if ((axis ? D.tile_begin_ax : D.tile_begin) != begin)
                    return fail(P, FDETD_E_ARG, "internal: tile ranges of the batch are not contiguous");
                for (int r = 0; r < nl; ++r) {
                    TileCoord c;
                    if (!decode_tile(D, r, halves, axis != 0, w, c) || c.i0 % w || c.k1 > D.nr)
                        return fail(P, FDETD_E_ARG, "internal: tile %d of a %dx%d grid leaves the grid", r, D.nz, D.nr);
                    const int u1 = std::min(units, (c.i0 + w) / kAxisColumns);
                    for (int u = c.i0 / kAxisColumns; u < u1; ++u)
                        for (int k = c.k0; k < c.k1; ++k)
                            if (seen[((size_t)c.half * units + u) * D.nr + k]++)
                                return fail(P, FDETD_E_ARG, "internal: a cell of a %dx%d grid is produced twice", D.nz, D.nr);
                }
            }
            for (unsigned char v : seen)
                if (v != 1) return fail(P, FDETD_E_ARG, "internal: a cell of a %dx%d grid is not produced", D.nz, D.nr);
        }
    for (const Batch &b : P->batches) {
        int n_main = 0, n_ax = 0;
        for (int t = 0; t < b.count; ++t) {
            const ProbDesc &D = P->desc[b.d0 + t];
            n_main += halves * D.nseg * D.nstrip;
            n_ax += halves * D.nseg_ax * D.nstrip_ax;
        }
        if (n_main != b.ntiles || n_ax != b.ntiles_ax) return fail(P, FDETD_E_ARG, "internal: tile count mismatch");
    }
    if (!P->ddesc) HIPCHK(P, hipMalloc(&P->ddesc, P->desc.size() * sizeof(ProbDesc)));
    HIPCHK(P, hipMemcpy(P->ddesc, P->desc.data(), P->desc.size() * sizeof(ProbDesc), hipMemcpyHostToDevice));
    return FDETD_OK;
}

// Arguments of one timing launch of batch b: a middle stage (the first when N < 3) with a current.  The
// stage vectors are the plan's own; psi and the current come from scratch[p] (np + 3 planes per problem,
// allocated for the tuning only), so that every operand is a separate stream of memory as in a real step.
BatchArgs tuning_args(fdetd_plan_t P, const Batch &b, const std::vector<void *> &scratch)
{
    BatchArgs A;
    std::memset(&A, 0, sizeof A);
    A.probs = P->ddesc + b.d0;
    A.nprob = b.count;
    A.N = b.N;
    A.n = b.N >= 3 ? b.N - 2 : b.N - 1;
    A.has_src = P->kind == FDETD_MAXWELL;
    A.compensated = P->precision == FDETD_FP32C;
    A.beta_in = -b.dt * std::ldexp(1.0, -b.N);
    A.beta = -b.dt * std::ldexp(1.0, -A.n);
    A.coef = b.dt / (A.n + 1);
    const size_t eb = elem_bytes(P->precision);
    const int np = planes(P->kind);
    for (int t = 0; t < b.count; ++t) {
        const int u = b.members[t];
        const size_t pb = P->probs[u].cells * eb;
        char *base = (char *)scratch[u];
        A.psi[t] = base;
        A.aux[t] = P->kind == FDETD_MAXWELL ? base + np * pb : base + pb;  // current, or a_tilde
        A.chi[t] = base + np * pb;
    }
    return A;
}

// Plan-time autotuning of the marching segment length: each launch batch runs a few timed stages at every
// candidate length (8 .. 256 rows) on tuning-only buffers and keeps the fastest.  The stage results do
// not depend on the tiling (every output is formed by the same operations in the same order), only the
// speed does.
int autotune(fdetd_plan_t P, double &ms_spent)
{
    ms_spent = 0.0;
    if ((P->flags & FDETD_PLAN_NO_AUTOTUNE) || forced_seg_rows()) return FDETD_OK;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t eb = elem_bytes(P->precision);
    const int np = planes(P->kind);
    // tuning-only psi and current (np + 3 planes per problem); without the memory the defaults stay
    std::vector<void *> scratch(P->probs.size(), nullptr);
    struct Free {
        std::vector<void *> &v;
        ~Free()
        {
            for (void *x : v)
                if (x) (void)hipFree(x);
        }
    } free_scratch{scratch};
    for (size_t u = 0; u < P->probs.size(); ++u) {
        const size_t bytes = (np + 3) * P->probs[u].cells * eb;
        if (hipMalloc(&scratch[u], bytes) != hipSuccess) {
            scratch[u] = nullptr;
            (void)hipGetLastError();
            return FDETD_OK;
        }
        HIPCHK(P, hipMemsetAsync(scratch[u], 0, bytes, P->stream));
    }
    for (const Prob &q : P->probs) {
        HIPCHK(P, hipMemsetAsync(q.buf[0], 0, np * q.cells * eb, P->stream));
        HIPCHK(P, hipMemsetAsync(q.buf[1], 0, np * q.cells * eb, P->stream));
        if (q.jbar) HIPCHK(P, hipMemsetAsync(q.jbar, 0, q.cells * eb, P->stream));
    }
    const size_t nb = P->batches.size();
    // rows a main launch of each batch marches over: longer candidates than the first one covering them
    // give the same tiling
    std::vector<int> rows(nb, 0);
    for (size_t bi = 0; bi < nb; ++bi)
        for (int t = 0; t < P->batches[bi].count; ++t) {
            const ProbDesc &D = P->desc[P->batches[bi].d0 + t];
            rows[bi] = std::max(rows[bi], D.nr - D.ax_rows);
        }
    // longer segments repay on tall grids and wide stencils (the window fill is 2 N_D - 1 rows per segment)
    static const int kCand[] = {8, 16, 32, 64, 128, 256};
    constexpr int kNC = 6;
    // candidate c of batch bi is timed unless a shorter candidate already covers the batch's rows
    auto distinct = [&](int ci, size_t bi) { return ci == 0 || kCand[ci - 1] < rows[bi]; };
    std::vector<double> t_ms(nb * kNC, 1e300);
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = FDETD_OK;
    hipError_t e = hipSuccess;
    if ((e = hipEventCreate(&ev[0])) || (e = hipEventCreate(&ev[1])))
        rc = fail(P, FDETD_E_HIP, "autotune: %s", hipGetErrorString(e));
    // two passes, ascending then descending, keeping each candidate's faster time
    for (int pass = 0; pass < 2 && !rc; ++pass)
        for (int k = 0; k < kNC && !rc; ++k) {
            const int ci = pass == 0 ? k : kNC - 1 - k;
            P->seg_rows.assign(nb, kCand[ci]);
            if ((rc = build_batches(P))) break;
            for (size_t bi = 0; bi < nb && !rc; ++bi) {
                if (!distinct(ci, bi)) continue;
                const Batch &b = P->batches[bi];
                BatchArgs A = tuning_args(P, b, scratch);
                constexpr int kReps = 4;
                for (int r = 0; r <= kReps && !rc; ++r) {  // one untimed launch, then kReps timed
                    if (r == 1 && (e = hipEventRecord(ev[0], P->stream)))
                        rc = fail(P, FDETD_E_HIP, "autotune: %s", hipGetErrorString(e));
                    if (!rc) rc = launch_stage(P, b, A, P->stream);
                }
                float ms = 0.f;
                if (!rc && ((e = hipEventRecord(ev[1], P->stream)) || (e = hipEventSynchronize(ev[1])) ||
                            (e = hipEventElapsedTime(&ms, ev[0], ev[1]))))
                    rc = fail(P, FDETD_E_HIP, "autotune: %s", hipGetErrorString(e));
                if (!rc) t_ms[bi * kNC + ci] = std::min(t_ms[bi * kNC + ci], (double)ms / kReps);
            }
        }
    std::vector<int> best(nb, kCand[0]);
    const bool log = std::getenv("FDETD_AUTOTUNE_LOG") != nullptr;  // per-candidate times on stderr
    for (size_t bi = 0; bi < nb; ++bi) {
        double bm = 1e300;
        for (int ci = 0; ci < kNC; ++ci)
            if (distinct(ci, bi) && t_ms[bi * kNC + ci] < bm) {
                bm = t_ms[bi * kNC + ci];
                best[bi] = kCand[ci];
            }
        if (log) {
            std::fprintf(stderr, "fdetd autotune batch %zu (N_D %d, %d problems):", bi, P->batches[bi].nd,
                         P->batches[bi].count);
            for (int ci = 0; ci < kNC; ++ci)
                if (distinct(ci, bi)) std::fprintf(stderr, " %d rows %.4f ms", kCand[ci], t_ms[bi * kNC + ci]);
            std::fprintf(stderr, " -> %d\n", best[bi]);
        }
    }
    if (!rc) {
        P->seg_rows = best;
        rc = build_batches(P);
    }
    // Store policy of the stage outputs and numbering of the tiles, at the chosen segment length: pairs of
    // consecutive stages (N - 2 and N - 3, each reading the other's output as in a step) under each of the
    // four combinations, two passes in opposite orders, the fastest kept.  Non-temporal outputs pay on grids
    // far larger than the caches and cost where the next stage would find them there; the tile numbering
    // changes which tiles share an XCD's L2 at a time; only timing tells.  FDETD_STORE_POLICY and
    // FDETD_TILE_ORDER fix either.
    if (!rc && P->kind == FDETD_MAXWELL && (forced_store_policy() < 0 || forced_tile_order() < 0)) {
        std::vector<double> tc(4 * nb, 1e300);
        for (int pass = 0; pass < 2 && !rc; ++pass)
            for (int k = 0; k < 4 && !rc; ++k) {
                const int combo = pass == 0 ? k : 3 - k;
                const int pol = combo & 1, ord = combo >> 1;
                if ((forced_store_policy() >= 0 && pol != forced_store_policy()) ||
                    (forced_tile_order() >= 0 && ord != forced_tile_order()))
                    continue;
                P->nt_store.assign(nb, pol);
                P->tile_order.assign(nb, ord);
                if ((rc = build_batches(P))) break;
                for (size_t bi = 0; bi < nb && !rc; ++bi) {
                    const Batch &b = P->batches[bi];
                    if (b.N < 4) continue;  // the pair needs two stages before the last
                    if (pol && !store_policy_applies(P, b)) continue;
                    BatchArgs A = tuning_args(P, b, scratch);
                    A.nt_store = pol;
                    constexpr int kPairs = 2;
                    for (int r = 0; r <= kPairs && !rc; ++r) {  // one untimed pair, then kPairs timed
                        if (r == 1 && (e = hipEventRecord(ev[0], P->stream)))
                            rc = fail(P, FDETD_E_HIP, "autotune: %s", hipGetErrorString(e));
                        for (int n = b.N - 2; n >= b.N - 3 && !rc; --n) {
                            A.n = n;
                            A.beta = -b.dt * std::ldexp(1.0, -n);
                            A.coef = b.dt / (n + 1);
                            rc = launch_stage(P, b, A, P->stream);
                        }
                    }
                    float ms = 0.f;
                    if (!rc && ((e = hipEventRecord(ev[1], P->stream)) || (e = hipEventSynchronize(ev[1])) ||
                                (e = hipEventElapsedTime(&ms, ev[0], ev[1]))))
                        rc = fail(P, FDETD_E_HIP, "autotune: %s", hipGetErrorString(e));
                    if (!rc) tc[4 * bi + combo] = std::min(tc[4 * bi + combo], (double)ms / (2 * kPairs));
                }
            }
        std::vector<int> pol_best(nb, std::max(0, forced_store_policy())), ord_best(nb, std::max(0, forced_tile_order()));
        for (size_t bi = 0; bi < nb && !rc; ++bi) {
            int cb = -1;
            for (int c = 0; c < 4; ++c)
                if (tc[4 * bi + c] < 1e299 && (cb < 0 || tc[4 * bi + c] < tc[4 * bi + cb])) cb = c;
            if (cb < 0) continue;  // not timed (Taylor order below 4): the defaults
            pol_best[bi] = cb & 1;
            ord_best[bi] = cb >> 1;
            if (log)
                std::fprintf(stderr, "fdetd autotune batch %zu store policy x tile order: %.4f / %.4f / %.4f / %.4f ms "
                             "(default, non-temporal; half first, segment first) -> %s, %s\n", bi, tc[4 * bi],
                             tc[4 * bi + 1], tc[4 * bi + 2], tc[4 * bi + 3], pol_best[bi] ? "non-temporal" : "default",
                             ord_best[bi] ? "segment first" : "half first");
        }
        if (!rc) {
            P->nt_store = pol_best;
            P->tile_order = ord_best;
            rc = build_batches(P);
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc) return rc;
    for (const Prob &q : P->probs)
        if (q.lo) HIPCHK(P, hipMemsetAsync(q.lo, 0, np * q.cells * 8, P->stream));
    ms_spent = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return FDETD_OK;
}

// Spectral radius of H by power iteration on -H^2 over a grid of at most 64 x 64 cells with the same
// mode, orders and spacings (the extreme eigenvectors live at the grid scale and near the axis, both
// present in the reduced grid).  FP64 arithmetic whatever the plan's precision: the estimate decides the
// time step a plan accepts (the norm of H grows with m, end of section 2.5).
int estimate_rho(fdetd_plan_t P, Prob &q, double &rho)
{
    Prob r = q;  // shares coefficients; own small buffers below
    r.d.nz = std::min(q.d.nz, 64);
    r.d.nr = std::min(q.d.nr, 64);
    r.cells = (size_t)r.d.nz * r.d.nr;
    const int prec = P64;
    const size_t eb = elem_bytes(FDETD_FP64);
    const int np = planes(P->kind);
    const size_t n = np * r.cells;
    void *x = nullptr, *t = nullptr, *y = nullptr, *zero = nullptr, *chi = nullptr;
    double *part = nullptr, *rp = nullptr, *rs = nullptr, *m2 = nullptr;
    const int nblk = 64;
    int rc = FDETD_OK;
    auto cleanup = [&]() {
        for (void *b : {x, t, y, zero, chi, (void *)part, (void *)rp, (void *)rs, (void *)m2})
            if (b) (void)hipFree(b);
    };
    do {
        hipError_t e = hipSuccess;
        if ((e = hipMalloc(&x, n * eb)) || (e = hipMalloc(&t, n * eb)) || (e = hipMalloc(&y, n * eb)) ||
            (e = hipMalloc(&zero, n * eb)) || (e = hipMalloc(&chi, r.cells * eb)) ||
            (e = hipMalloc(&part, nblk * sizeof(double))) || (e = hipMalloc(&rp, r.d.nr * sizeof(double))) ||
            (e = hipMalloc(&rs, r.d.nr * sizeof(double))) || (e = hipMalloc(&m2, r.d.nr * sizeof(double)))) {
            rc = fail(P, FDETD_E_NOMEM, "stability estimate: %s", hipGetErrorString(e));
            break;
        }
        std::vector<double> hr(r.d.nr), hs(r.d.nr), hm(r.d.nr);
        for (int k = 0; k < r.d.nr; ++k) {
            const double rho_k = (k + 0.5) * r.d.dr;
            hr[k] = 1.0 / rho_k;
            hs[k] = k ? 1.0 / (k * r.d.dr) : 0.0;
            hm[k] = (double)r.d.m * r.d.m / (rho_k * rho_k);
        }
        if (hipMemcpy(rp, hr.data(), r.d.nr * 8, hipMemcpyHostToDevice) ||
            hipMemcpy(rs, hs.data(), r.d.nr * 8, hipMemcpyHostToDevice) ||
            hipMemcpy(m2, hm.data(), r.d.nr * 8, hipMemcpyHostToDevice) || hipMemset(zero, 0, n * eb) ||
            hipMemset(chi, 0, r.cells * eb)) {
            rc = fail(P, FDETD_E_HIP, "stability estimate: copy failed");
            break;
        }
        r.rinv_p = rp;
        r.rinv_s = rs;
        r.m2rinv2 = m2;
        // deterministic pseudo-random start vector (splitmix64 stream)
        std::vector<double> h(2 * n);
        uint64_t st = 0x9E3779B97F4A7C15ull ^ (uint64_t)q.d.m;
        for (auto &v : h) {
            uint64_t z = (st += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            v = (double)(z >> 11) * 0x1.0p-53 - 0.5;
        }
        if (hipMemcpy(x, h.data(), n * 16, hipMemcpyHostToDevice)) {
            rc = fail(P, FDETD_E_HIP, "stability estimate: copy failed");
            break;
        }
        auto applyH = [&](const void *in, void *out) -> int {
            if (P->kind == FDETD_MAXWELL) {
                MaxwellStageArgs A;
                fill_maxwell_args(P, r, A);
                A.vin = in;
                A.psi = zero;
                A.vout = out;
                A.coef = 1.0;
                HIPCHK(P, launch_maxwell_stage(prec, r.nd, A, P->stream));
            } else {
                EnvelopeStageArgs A;
                fill_envelope_args(P, r, A);
                A.vin_a = in;
                A.vin_t = (const char *)in + r.cells * eb;
                A.psi_a = zero;
                A.psi_t = zero;
                A.chi = chi;
                A.out_a = out;
                A.out_t = (char *)out + r.cells * eb;
                A.coef = 1.0;
                HIPCHK(P, launch_envelope_stage(prec, r.nd, A, P->stream));
            }
            return FDETD_OK;
        };
        auto norm = [&](const void *v, double &out) -> int {
            HIPCHK(P, launch_norm2(prec, v, n, part, nblk, P->stream));
            std::vector<double> hp(nblk);
            HIPCHK(P, hipMemcpyAsync(hp.data(), part, nblk * sizeof(double), hipMemcpyDeviceToHost, P->stream));
            HIPCHK(P, hipStreamSynchronize(P->stream));
            out = 0.0;
            for (double v2 : hp) out += v2;
            out = std::sqrt(out);
            return FDETD_OK;
        };
        double nx = 0.0;
        if ((rc = norm(x, nx))) break;
        HIPCHK(P, launch_scale(prec, x, n, 1.0 / nx, P->stream));
        double lam = 0.0;
        for (int it = 0; it < 60 && rc == FDETD_OK; ++it) {
            if ((rc = applyH(x, t)) || (rc = applyH(t, y))) break;
            double ny = 0.0;
            if ((rc = norm(y, ny))) break;
            lam = ny;  // |H^2 x| with |x| = 1
            if (!(ny > 0.0) || !std::isfinite(ny)) break;
            HIPCHK(P, launch_scale(prec, y, n, 1.0 / ny, P->stream));
            std::swap(x, y);
        }
        rho = std::sqrt(lam);
    } while (0);
    (void)hipStreamSynchronize(P->stream);
    cleanup();
    return rc;
}

int validate(const fdetd_problem_desc &d, int idx)
{
    const int nd = d.fd_order / 2;
    if (d.kind != FDETD_MAXWELL && d.kind != FDETD_ENVELOPE)
        return fail(nullptr, FDETD_E_ARG, "problem %d: unknown kind %d", idx, d.kind);
    if (d.fd_order < 2 || d.fd_order > 2 * kMaxND || (d.fd_order & 1))
        return fail(nullptr, FDETD_E_ARG, "problem %d: fd_order %d not even in [2, 32]", idx, d.fd_order);
    if (d.nz < 2 * nd + 1 || d.nr < nd + 1)
        return fail(nullptr, FDETD_E_ARG, "problem %d: grid %d x %d too small for order %d (need nz >= %d, nr >= %d)",
                    idx, d.nz, d.nr, d.fd_order, 2 * nd + 1, nd + 1);
    if ((int64_t)d.nz * d.nr > (int64_t)1 << 31)
        return fail(nullptr, FDETD_E_ARG, "problem %d: more than 2^31 cells", idx);
    if (d.m < 0 || d.m > 64) return fail(nullptr, FDETD_E_ARG, "problem %d: mode %d not in [0, 64]", idx, d.m);
    if (d.taylor_order < 1 || d.taylor_order > 32)
        return fail(nullptr, FDETD_E_ARG, "problem %d: taylor_order %d not in [1, 32]", idx, d.taylor_order);
    if (!(d.dz > 0) || !(d.dr > 0) || !(d.dt > 0) || !std::isfinite(d.dz + d.dr + d.dt))
        return fail(nullptr, FDETD_E_ARG, "problem %d: dz, dr, dt must be finite and > 0", idx);
    if (d.kind == FDETD_ENVELOPE && !std::isfinite(d.k0))
        return fail(nullptr, FDETD_E_ARG, "problem %d: k0 not finite", idx);
    return FDETD_OK;
}

// Non-null and aligned to a bytes (the element: complex 16 B FP64 / 8 B FP32C, real 8 / 4 B).
bool aligned(const void *p, size_t a) { return p && ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" {

int fdetd_coefficients(int32_t which, int32_t nd, double *out)
{
    if (!out || !make_coefficients(which, nd, out))
        return fail(nullptr, FDETD_E_ARG, "fdetd_coefficients: bad table %d or nd %d", which, nd);
    return FDETD_OK;
}

double fdetd_taylor_stability_bound(int32_t taylor_order) { return taylor_stability_bound(taylor_order); }

const char *fdetd_last_error(fdetd_plan_t plan) { return plan ? plan->err.c_str() : g_last_error.c_str(); }

void fdetd_destroy(fdetd_plan_t plan)
{
    if (!plan) return;
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    for (hipStream_t s : plan->lanes) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : plan->join_ev) (void)hipEventDestroy(e);
    if (plan->fork_ev) (void)hipEventDestroy(plan->fork_ev);
    if (plan->axis_stream) {
        (void)hipStreamSynchronize(plan->axis_stream);
        (void)hipStreamDestroy(plan->axis_stream);
    }
    if (plan->axis_fork) (void)hipEventDestroy(plan->axis_fork);
    if (plan->axis_join) (void)hipEventDestroy(plan->axis_join);
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
    for (auto &q : plan->probs) free_prob(q);
    if (plan->zero) (void)hipFree(plan->zero);
    if (plan->ddesc) (void)hipFree(plan->ddesc);
    delete plan;
}

int fdetd_plan(const fdetd_problem_desc *probs, int32_t n_probs, int32_t precision, uint32_t flags,
               void *stream, fdetd_plan_t *out)
{
    if (!out) return fail(nullptr, FDETD_E_ARG, "fdetd_plan: out is NULL");
    *out = nullptr;
    if (!probs || n_probs < 1) return fail(nullptr, FDETD_E_ARG, "fdetd_plan: need at least one problem");
    if (precision != FDETD_FP64 && precision != FDETD_FP32C)
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: unknown precision %d", precision);
    for (int p = 0; p < n_probs; ++p) {
        int rc = validate(probs[p], p);
        if (rc) return rc;
        if (probs[p].kind != probs[0].kind)
            return fail(nullptr, FDETD_E_ARG, "fdetd_plan: all problems of a plan must have the same kind");
    }
    if (flags & ~(FDETD_PLAN_SEPARATE_WN * 2u - 1u))
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: unknown flag bits 0x%x", flags & ~(FDETD_PLAN_SEPARATE_WN * 2u - 1u));
    if ((flags & FDETD_PLAN_INCREMENT_FORM) && precision != FDETD_FP32C)
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: FDETD_PLAN_INCREMENT_FORM needs an FP32C plan");
    if ((flags & FDETD_PLAN_USE_GRAPH) && !stream)
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: graph capture needs a non-default stream");
    if ((flags & FDETD_PLAN_CURRENT_CORRECTION) && probs[0].kind != FDETD_MAXWELL)
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: the current correction needs Maxwell problems");
    if ((flags & FDETD_PLAN_USE_GRAPH) && (flags & FDETD_PLAN_PROFILE))
        return fail(nullptr, FDETD_E_ARG, "fdetd_plan: FDETD_PLAN_PROFILE times eager launches only");
    fdetd_plan_t P = new (std::nothrow) fdetd_plan_s;
    if (!P) return fail(nullptr, FDETD_E_NOMEM, "fdetd_plan: host allocation failed");
    P->precision = precision;
    P->flags = flags;
    P->kind = probs[0].kind;
    P->stream = (hipStream_t)stream;
    P->probs.resize(n_probs);
    const size_t eb = elem_bytes(precision);
    const int np = planes(P->kind);
    int64_t scratch = 0, bytes_step = 0, cells = 0, launches = 0;
    double worst = 0.0, margin = 0.0;
    int rc = FDETD_OK;
    for (int p = 0; p < n_probs && rc == FDETD_OK; ++p) {
        Prob &q = P->probs[p];
        q.d = probs[p];
        q.nd = q.d.fd_order / 2;
        q.cells = (size_t)q.d.nz * q.d.nr;
        make_coefficients(COEF_STAGGERED, q.nd, q.a);
        make_coefficients(COEF_HALFSHIFT, q.nd, q.s);
        make_coefficients(COEF_CENTRED_D1, q.nd, q.d1);
        make_coefficients(COEF_CENTRED_D2, q.nd, q.d2);
        make_coefficients(COEF_AXIS, q.nd, q.c);
        hipError_t e = hipSuccess;
        const size_t vec_b = np * q.cells * eb;
        if ((e = hipMalloc(&q.buf[0], vec_b)) || (e = hipMalloc(&q.buf[1], vec_b)) ||
            (P->kind == FDETD_MAXWELL && (e = hipMalloc(&q.jbar, q.cells * eb))) ||
            (precision == FDETD_FP32C && (e = hipMalloc((void **)&q.lo, np * q.cells * sizeof(float) * 2))) ||
            (e = hipMalloc((void **)&q.rinv_p, q.d.nr * sizeof(double))) ||
            (e = hipMalloc((void **)&q.rinv_s, q.d.nr * sizeof(double))) ||
            (e = hipMalloc((void **)&q.m2rinv2, q.d.nr * sizeof(double))) ||
            (P->kind == FDETD_ENVELOPE && ((e = hipMalloc((void **)&q.sz, q.d.nz * sizeof(double))) ||
                                           (e = hipMalloc((void **)&q.sr, q.d.nr * sizeof(double))))) ||
            ((flags & FDETD_PLAN_INCREMENT_FORM) && (e = hipMalloc(&q.pbuf, np * q.cells * 8)))) {
            rc = fail(P, e == hipErrorOutOfMemory ? FDETD_E_NOMEM : FDETD_E_HIP, "fdetd_plan: problem %d: %s", p,
                      hipGetErrorString(e));
            break;
        }
        scratch += 2 * vec_b + (P->kind == FDETD_MAXWELL ? q.cells * eb : 0) +
                   (precision == FDETD_FP32C ? np * q.cells * 8 : 0) + 3 * q.d.nr * 8 +
                   (P->kind == FDETD_ENVELOPE ? (q.d.nz + q.d.nr) * 8 : 0) +
                   ((flags & FDETD_PLAN_INCREMENT_FORM) ? np * q.cells * 8 : 0);
        std::vector<double> hr(q.d.nr), hs(q.d.nr), hm(q.d.nr);
        for (int k = 0; k < q.d.nr; ++k) {
            const double rho_k = (k + 0.5) * q.d.dr;
            hr[k] = 1.0 / rho_k;
            hs[k] = k ? 1.0 / (k * q.d.dr) : 0.0;
            hm[k] = (double)q.d.m * q.d.m / (rho_k * rho_k);
        }
        if ((e = hipMemcpy(q.rinv_p, hr.data(), q.d.nr * 8, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(q.rinv_s, hs.data(), q.d.nr * 8, hipMemcpyHostToDevice)) ||
            (e = hipMemcpy(q.m2rinv2, hm.data(), q.d.nr * 8, hipMemcpyHostToDevice)) ||
            (precision == FDETD_FP32C && (e = hipMemset(q.lo, 0, np * q.cells * 8))) ||
            (q.sz && (e = hipMemset(q.sz, 0, q.d.nz * sizeof(double)))) ||
            (q.sr && (e = hipMemset(q.sr, 0, q.d.nr * sizeof(double))))) {
            rc = fail(P, FDETD_E_HIP, "fdetd_plan: problem %d: %s", p, hipGetErrorString(e));
            break;
        }
        if (P->kind == FDETD_MAXWELL && (flags & FDETD_PLAN_CURRENT_CORRECTION)) {
            std::vector<double> band;
            if (!radial_lu(q, band)) {
                rc = fail(P, FDETD_E_ARG, "fdetd_plan: problem %d: the radial operator of the current correction is singular", p);
                break;
            }
            // segments of the partitioned solve: at least 2 nd rows, at most about 8 segments
            q.seg = std::max(2 * q.nd, (q.d.nr + 7) / 8);
            q.nseg = (q.d.nr + q.seg - 1) / q.seg;
            std::vector<double> gresp;
            segment_responses(q, band, q.seg, gresp);
            if ((e = hipMalloc((void **)&q.band, band.size() * sizeof(double))) || (e = hipMalloc(&q.jth, q.cells * eb)) ||
                (e = hipMalloc((void **)&q.gresp, gresp.size() * sizeof(double))) ||
                (e = hipMemcpy(q.band, band.data(), band.size() * sizeof(double), hipMemcpyHostToDevice)) ||
                (e = hipMemcpy(q.gresp, gresp.data(), gresp.size() * sizeof(double), hipMemcpyHostToDevice))) {
                rc = fail(P, e == hipErrorOutOfMemory ? FDETD_E_NOMEM : FDETD_E_HIP, "fdetd_plan: problem %d: %s", p,
                          hipGetErrorString(e));
                break;
            }
            scratch += (band.size() + gresp.size()) * sizeof(double) + q.cells * eb;
            // div: read Jbar_rho, J_theta, rho_xy, write d; solve: d, y, y, phi (FP64); apply: read phi, Jbar_rho,
            // J_theta, write Jbar_rho, J_theta~
            bytes_step += (int64_t)q.cells * (8 * eb + 5 * 16);
        }
        const int N = q.d.taylor_order;
        cells += q.cells;
        if (P->kind == FDETD_MAXWELL) {
            // per stage: read v, psi (6c each), Jbar (3c), write v (6c); staging J_rho: 2c; FP32C: lo r+w.
            // (Forming w_N -- in the first stage, 3c more, or in a pass of its own, 9c -- is not counted:
            // it is an implementation overhead of the first stage.)
            bytes_step += (int64_t)q.cells * eb * (21 * N + 2) + (precision == FDETD_FP32C ? q.cells * 6 * 8 * 2 : 0);
            // increment form: P = H lo (zeros, lo, P: 18c), P += H psi (psi, P, P: 18c); the last stage also
            // reads psi (6c)
            if (flags & FDETD_PLAN_INCREMENT_FORM) bytes_step += (int64_t)q.cells * eb * 42;
            // (staging, w_N, stage and axis-rule launches are counted per batch below)
        } else {
            // per stage: read v (2c), psi (2c), chi (1 real), write v (2c)
            bytes_step += (int64_t)q.cells * (eb * 6 + eb / 2) * N + (precision == FDETD_FP32C ? q.cells * 2 * 8 * 2 : 0);
            // increment form: two P passes (6c + chi each) and psi_hi in the last stage (2c)
            if (flags & FDETD_PLAN_INCREMENT_FORM) bytes_step += (int64_t)q.cells * (eb * 14 + eb);
        }
        if (!(flags & FDETD_PLAN_SKIP_STABILITY)) {
            double rho = 0.0;
            if ((rc = estimate_rho(P, q, rho))) break;
            q.rho_hat = rho;
            const double xn = taylor_stability_bound(N);
            const double x = q.d.dt * rho;
            worst = std::max(worst, x);
            const double mg = x > 0 ? xn / x : 1e300;
            margin = (p == 0) ? mg : std::min(margin, mg);
            if (x * 1.02 >= xn) {
                rc = fail(P, FDETD_E_UNSTABLE,
                          "problem %d: dt * rho(H) = %.4f (rho estimated %.6g) exceeds the Taylor order-%d bound %.4f / 1.02",
                          p, x, rho, N, xn);
                break;
            }
        }
    }
    if (rc == FDETD_OK && (flags & FDETD_PLAN_INCREMENT_FORM)) {
        size_t zb = 0;
        for (const Prob &q : P->probs) zb = std::max(zb, 6 * q.cells * 8);
        hipError_t e = hipSuccess;
        if ((e = hipMalloc(&P->zero, zb)) || (e = hipMemset(P->zero, 0, zb)))
            rc = fail(P, e == hipErrorOutOfMemory ? FDETD_E_NOMEM : FDETD_E_HIP, "fdetd_plan: %s", hipGetErrorString(e));
        scratch += zb;
    }
    if (rc == FDETD_OK) rc = build_batches(P);
    double tune_ms = 0.0;
    if (rc == FDETD_OK) rc = autotune(P, tune_ms);
    if (rc == FDETD_OK) rc = assign_lanes(P);
    if (rc == FDETD_OK) rc = make_axis_stream(P);
    if (rc != FDETD_OK) {
        g_last_error = P->err;
        fdetd_destroy(P);
        return rc;
    }
    P->info.n_probs = n_probs;
    P->info.precision = precision;
    P->info.dt_rho_max = worst;
    P->info.stability_margin = margin;
    P->info.cells = cells;
    P->info.bytes_per_step = bytes_step;
    P->info.scratch_bytes = scratch;
    for (const Batch &b : P->batches) {  // Maxwell: N stages (two launches each when a batch that mixes
                                         // widths has FP32C near-axis tiles), staging and w_N per batch
        const int per_stage = (b.nd < 0 && b.ntiles && b.ntiles_ax) ? 2 : 1;
        const int prepass = (flags & FDETD_PLAN_INCREMENT_FORM) ? 2 : 0;  // the two P passes
        const int staging = P->kind == FDETD_MAXWELL ? (fuse_wn(P, b, true) ? 1 : 2) : 0;  // J_rho, w_N
        launches += (int64_t)(per_stage * b.N + staging + prepass) * (b.ntiles + b.ntiles_ax > 0);
    }
    P->info.launches_per_step = launches;
    P->info.seg_rows = P->batches.empty() ? 0 : P->batches[0].seg;
    P->info.seg_rows_axis = P->desc.empty() ? 0 : P->desc[0].seg_ax;
    P->info.store_policy = P->batches.empty() ? 0 : P->batches[0].nt_store;
    P->info.tile_order = P->batches.empty() ? 0 : P->batches[0].tile_order;
    P->info.autotune_ms = tune_ms;
    P->info.streams = 1 + (int32_t)P->lanes.size();
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        fail(P, FDETD_E_HIP, "fdetd_plan: %s", hipGetErrorString(e));
        g_last_error = P->err;
        fdetd_destroy(P);
        return FDETD_E_HIP;
    }
    *out = P;
    return FDETD_OK;
}

int fdetd_deposit_jz(fdetd_plan_t plan, const double *samples, int64_t n, double vz, double eps,
                     void *const *j_half)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_deposit_jz: NULL plan");
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_deposit_jz: plan is not a Maxwell plan");
    if (n < 0 || !j_half || (n > 0 && !aligned(samples, 8)) || !(eps >= 0.0 && eps <= 1.0) || !std::isfinite(vz))
        return fail(plan, FDETD_E_ARG, "fdetd_deposit_jz: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        if (!aligned(j_half[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_deposit_jz: j_half[%zu] NULL or not %zu-byte aligned", p, eb);
    }
    if (n == 0) return FDETD_OK;
    for (const Batch &b : plan->batches) {
        DepositArgs A;
        std::memset(&A, 0, sizeof A);
        A.probs = plan->ddesc + b.d0;
        A.nprob = b.count;
        A.n = n;
        A.samples = samples;
        A.vz = vz;
        A.eps = eps;
        for (int t = 0; t < b.count; ++t) A.j[t] = j_half[b.members[t]];
        HIPCHK(plan, launch_deposit_jz(prec_code(plan->precision), A, plan->stream));
    }
    return FDETD_OK;
}

int fdetd_deposit_current(fdetd_plan_t plan, const double *samples, int64_t n, double eps, void *const *j_half)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_deposit_current: NULL plan");
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_deposit_current: plan is not a Maxwell plan");
    if (n < 0 || !j_half || (n > 0 && !aligned(samples, 8)) || !(eps >= 0.0 && eps <= 1.0))
        return fail(plan, FDETD_E_ARG, "fdetd_deposit_current: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p)
        if (!aligned(j_half[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_deposit_current: j_half[%zu] NULL or not %zu-byte aligned", p, eb);
    if (n == 0) return FDETD_OK;
    for (const Batch &b : plan->batches) {
        DepositArgs A;
        std::memset(&A, 0, sizeof A);
        A.probs = plan->ddesc + b.d0;
        A.nprob = b.count;
        A.n = n;
        A.samples = samples;
        A.eps = eps;
        A.rho_xy = (plan->flags & FDETD_PLAN_CURRENT_CORRECTION) != 0;
        for (int t = 0; t < b.count; ++t) A.j[t] = j_half[b.members[t]];
        HIPCHK(plan, launch_deposit_current(prec_code(plan->precision), A, plan->stream));
    }
    return FDETD_OK;
}

int fdetd_deposit_rho(fdetd_plan_t plan, const double *samples, int64_t n, double dz_shift, double eps,
                      void *const *rho)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_deposit_rho: NULL plan");
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_deposit_rho: plan is not a Maxwell plan");
    if (n < 0 || !rho || (n > 0 && !aligned(samples, 8)) || !(eps >= 0.0 && eps <= 1.0) || !std::isfinite(dz_shift))
        return fail(plan, FDETD_E_ARG, "fdetd_deposit_rho: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p)
        if (!aligned(rho[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_deposit_rho: rho[%zu] NULL or not %zu-byte aligned", p, eb);
    if (n == 0) return FDETD_OK;
    for (const Batch &b : plan->batches) {
        DepositArgs A;
        std::memset(&A, 0, sizeof A);
        A.probs = plan->ddesc + b.d0;
        A.nprob = b.count;
        A.n = n;
        A.samples = samples;
        A.shift = dz_shift;
        A.eps = eps;
        for (int t = 0; t < b.count; ++t) A.j[t] = rho[b.members[t]];
        HIPCHK(plan, launch_deposit_rho(prec_code(plan->precision), A, plan->stream));
    }
    return FDETD_OK;
}

namespace {
int gather_impl(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields, int ss);
int gather_supersampled(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields,
                        int ss, int *box);
}

int fdetd_gather_supersampled(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n,
                              double *fields, int32_t supersample)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_gather_supersampled: NULL plan");
    if (supersample < 0 || supersample > 3)
        return fail(plan, FDETD_E_ARG, "fdetd_gather_supersampled: supersample %d not in 0..3", supersample);
    return gather_impl(plan, psi, samples, n, fields, supersample);
}

int fdetd_gather(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_gather: NULL plan");
    return gather_impl(plan, psi, samples, n, fields, 0);
}

namespace {
int gather_impl(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields, int ss)
{
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_gather: plan is not a Maxwell plan");
    const int np = (int)plan->probs.size();
    if (!psi || n < 0 || (n > 0 && (!aligned(samples, 8) || !aligned(fields, 8))))
        return fail(plan, FDETD_E_ARG, "fdetd_gather: bad arguments");
    if (np > kMaxGather) return fail(plan, FDETD_E_ARG, "fdetd_gather: at most %d problems (modes of one grid)", kMaxGather);
    const size_t eb = elem_bytes(plan->precision);
    const fdetd_problem_desc &d0 = plan->probs[0].d;
    for (int p = 0; p < np; ++p) {
        const fdetd_problem_desc &d = plan->probs[p].d;
        if (d.nz != d0.nz || d.nr != d0.nr || d.dz != d0.dz || d.dr != d0.dr)
            return fail(plan, FDETD_E_ARG, "fdetd_gather: problem %d is not a mode of the same grid as problem 0", p);
        if (!aligned(psi[p], eb)) return fail(plan, FDETD_E_ARG, "fdetd_gather: psi[%d] NULL or misaligned", p);
    }
    if (ss != 0 && 4 * plan->probs[0].cells > (size_t)INT32_MAX)
        return fail(plan, FDETD_E_ARG, "fdetd_gather_supersampled: grid of %zu cells too large (at most 2^29)",
                    plan->probs[0].cells);
    if (n == 0) return FDETD_OK;
    const int prec = prec_code(plan->precision);
    // The nodes and rows the samples' shapes touch: the destagger passes compute only those (rows grown
    // where a later pass reads more).  The box and the partial boxes of its reduction sit in planes 1..5
    // of problem 0's second stage vector, which the gather does not otherwise use.
    const size_t pb0 = plan->probs[0].cells * elem_bytes(plan->precision);
    int *box = (int *)((char *)plan->probs[0].buf[1] + pb0);
    const size_t room = (5 * pb0) / (4 * sizeof(int)) - 1;
    HIPCHK(plan, launch_gather_box(samples, n, d0.nz, d0.nr, d0.dz, d0.dr, box, box + 4,
                                   (int)std::min<size_t>(room, 2048), plan->stream));
    if (ss != 0) return gather_supersampled(plan, psi, samples, n, fields, ss, box);
    GatherArgs G;
    std::memset(&G, 0, sizeof G);
    G.n = n;
    G.samples = samples;
    G.fields = fields;
    G.nprob = np;
    G.nz = d0.nz;
    G.nr = d0.nr;
    G.dz = d0.dz;
    G.dr = d0.dr;
    // Destaggered components go to buf[0] (E_theta is read from psi); B_theta's z shift goes to buf[1] and
    // its rho pass reads that, so it runs in the next launch, beside the independent passes of the next
    // problem: np + 1 launches in all.
    DestaggerArgs X;
    std::memset(&X, 0, sizeof X);
    X.nz = d0.nz;
    X.nr = d0.nr;
    X.box = box;
    auto coeffs = [&](int set, const Prob &q) {
        X.nd[set] = q.nd;
        for (int j = 0; j < q.nd; ++j) {
            X.s[set][j] = q.s[j];
            X.c[set][j] = q.c[j];
        }
    };
    auto plane = [&](const Prob &q, const void *base, int c) {
        return (void *)((const char *)base + c * q.cells * eb);
    };
    auto parities = [](int m, int &pS, int &pA) {
        pS = (m % 2 == 0) ? 1 : -1;
        pA = (std::abs(m - 1) % 2 == 0) ? 1 : -1;
    };
    for (int p = 0; p <= np; ++p) {
        X.npass = 0;
        auto add = [&](const void *src, void *dst, int rho, int parity, int extrapolate, int grow_r, int set) {
            X.pass[X.npass++] = DestaggerPass{src, dst, rho, parity, extrapolate, 0, grow_r, set};
        };
        if (p > 0) {  // B_theta's rho pass of the previous problem
            const Prob &q = plan->probs[p - 1];
            int pS, pA;
            parities(q.d.m, pS, pA);
            coeffs(1, q);
            add(plane(q, q.buf[1], 0), plane(q, q.buf[0], BTH), 1, pA, q.d.m == 1, 0, 1);
        }
        if (p < np) {
            const Prob &q = plan->probs[p];
            int pS, pA;
            parities(q.d.m, pS, pA);
            coeffs(0, q);
            add(plane(q, psi[p], ER), plane(q, q.buf[0], ER), 1, pA, q.d.m == 1, 0, 0);
            add(plane(q, psi[p], EZ), plane(q, q.buf[0], EZ), 0, 1, 0, 0, 0);
            add(plane(q, psi[p], BR), plane(q, q.buf[0], BR), 0, 1, 0, 0, 0);
            add(plane(q, psi[p], BTH), plane(q, q.buf[1], 0), 0, 1, 0, q.nd, 0);  // read at +-nd rows next
            add(plane(q, psi[p], BZ), plane(q, q.buf[0], BZ), 1, pS, q.d.m == 0, 0, 0);
            G.m[p] = q.d.m;
            for (int c = 0; c < 6; ++c) G.plane[p][c] = c == ETH ? plane(q, psi[p], ETH) : plane(q, q.buf[0], c);
        }
        HIPCHK(plan, launch_destagger(prec, X, plan->stream));
    }
    HIPCHK(plan, launch_gather(prec, G, plan->stream));
    return FDETD_OK;
}

// 2x supersampling: for each component the position sets (zs, rs) the doubled grid needs (zs over {0, 1}
// when z is doubled, else {0}; rs likewise), each made from the stored set by at most one half shift along
// z followed by one along rho, all in the plan's doubled-grid planes (the stored set copied there).  Level
// 1 shifts and copies the stored planes (z shifts computed on rows grown by N_D, which the level-2 rho
// shifts and axis rows read); level 2 shifts level 1's z output along rho and sets its axis row.  Level 2
// of problem p - 1 shares a launch with level 1 of problem p.
int gather_supersampled(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields,
                        int ss, int *box)
{
    const int np = (int)plan->probs.size();
    const size_t eb = elem_bytes(plan->precision);
    const int prec = prec_code(plan->precision);
    const fdetd_problem_desc &d0 = plan->probs[0].d;
    for (int p = 0; p < np; ++p) {
        Prob &q = plan->probs[p];
        if (!q.fine && hipMalloc(&q.fine, 24 * q.cells * eb) != hipSuccess) {
            q.fine = nullptr;
            (void)hipGetLastError();
            return fail(plan, FDETD_E_NOMEM, "fdetd_gather_supersampled: no memory for the doubled grids");
        }
    }
    static const int own_z[6] = {0, 0, 1, 1, 1, 0}, own_r[6] = {1, 0, 0, 0, 1, 1};
    const bool dz2 = ss & 1, dr2 = ss & 2;
    auto needed = [&](int zs, int rs) { return (zs == 0 || dz2) && (rs == 0 || dr2); };
    DestaggerArgs X;
    std::memset(&X, 0, sizeof X);
    X.nz = d0.nz;
    X.nr = d0.nr;
    X.box = box;
    auto coeffs = [&](int set, const Prob &q) {
        X.nd[set] = q.nd;
        for (int j = 0; j < q.nd; ++j) {
            X.s[set][j] = q.s[j];
            X.c[set][j] = q.c[j];
        }
    };
    for (int p = 0; p <= np; ++p) {
        X.npass = 0;
        for (int lvl = 2; lvl >= 1; --lvl) {
            const int pp = lvl == 2 ? p - 1 : p, set = lvl == 2 ? 1 : 0;
            if (pp < 0 || pp >= np) continue;
            const Prob &q = plan->probs[pp];
            coeffs(set, q);
            const int m = q.d.m, pS = (m % 2 == 0) ? 1 : -1, pA = (std::abs(m - 1) % 2 == 0) ? 1 : -1;
            const size_t pb = q.cells * eb;
            auto fine = [&](int c, int zs, int rs) { return (void *)((char *)q.fine + (4 * c + zs + 2 * rs) * pb); };
            for (int c = 0; c < 6; ++c) {
                const int zn = own_z[c], rn = own_r[c], par = (c == EZ || c == BZ) ? pS : pA;
                const int ext = (c == ER || c == BTH) ? m == 1 : (c == BZ ? m == 0 : 0);
                const void *stored = (const char *)psi[pp] + c * pb;
                auto add = [&](const void *src, void *dst, int op, int to_stag, int grow_r, int axis_rule) {
                    X.pass[X.npass++] = DestaggerPass{src, dst, op, par, op != PASS_Z ? ext : 0, to_stag, grow_r, set,
                                                      axis_rule};
                };
                if (lvl == 1) {
                    if (needed(1 - zn, 0) || needed(1 - zn, 1))
                        add(stored, fine(c, 1 - zn, rn), PASS_Z, zn == 0, q.nd, 0);
                    if (needed(zn, 1 - rn)) add(stored, fine(c, zn, 1 - rn), PASS_RHO, rn == 0, 0, 0);
                    if (needed(zn, rn)) add(stored, fine(c, zn, rn), PASS_COPY, 0, 0, rn == 1);
                } else {
                    if (needed(1 - zn, 1 - rn)) add(fine(c, 1 - zn, rn), fine(c, 1 - zn, 1 - rn), PASS_RHO, rn == 0, 0, 0);
                    // the z-shifted staggered-rho set: its axis row by the axis rule (the rho pass above
                    // does not read that row)
                    if (rn == 1 && needed(1 - zn, 1)) add(fine(c, 1 - zn, 1), fine(c, 1 - zn, 1), PASS_AXIS, 0, 0, 1);
                }
            }
        }
        HIPCHK(plan, launch_destagger(prec, X, plan->stream));
    }
    GatherArgs G;
    std::memset(&G, 0, sizeof G);
    G.n = n;
    G.samples = samples;
    G.fields = fields;
    G.nprob = np;
    G.nz = d0.nz;
    G.nr = d0.nr;
    G.dz = d0.dz;
    G.dr = d0.dr;
    G.ss = ss;
    G.plane_bytes = plan->probs[0].cells * eb;
    for (int p = 0; p < np; ++p) {
        G.m[p] = plan->probs[p].d.m;
        G.fine[p] = plan->probs[p].fine;
    }
    HIPCHK(plan, launch_gather(prec, G, plan->stream));
    return FDETD_OK;
}
}  // namespace

int envelope_ponderomotive(fdetd_plan_t plan, const void *const *a, void *const *out)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "envelope_ponderomotive: NULL plan");
    if (plan->kind != FDETD_ENVELOPE) return fail(plan, FDETD_E_ARG, "envelope_ponderomotive: plan is not an envelope plan");
    if (!a || !out) return fail(plan, FDETD_E_ARG, "envelope_ponderomotive: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        if (plan->probs[p].d.m != 0)
            return fail(plan, FDETD_E_ARG, "envelope_ponderomotive: problem %zu has m = %d (needs m = 0)", p,
                        plan->probs[p].d.m);
        if (!aligned(a[p], eb) || !aligned(out[p], eb / 2))
            return fail(plan, FDETD_E_ARG, "envelope_ponderomotive: pointer of problem %zu NULL or misaligned", p);
    }
    for (const Batch &b : plan->batches)
        for (int t = 0; t < b.count; ++t) {
            const int p = b.members[t];
            const Prob &q = plan->probs[p];
            HIPCHK(plan, launch_ponderomotive(prec_code(plan->precision), plan->ddesc + b.d0 + t, q.d.nz, q.d.nr, q.nd,
                                              a[p], out[p], plan->stream));
        }
    return FDETD_OK;
}

int envelope_gather(fdetd_plan_t plan, int32_t problem, const void *pond, const double *samples, int64_t n,
                    double *out)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "envelope_gather: NULL plan");
    if (plan->kind != FDETD_ENVELOPE) return fail(plan, FDETD_E_ARG, "envelope_gather: plan is not an envelope plan");
    if (problem < 0 || problem >= (int)plan->probs.size())
        return fail(plan, FDETD_E_ARG, "envelope_gather: problem %d out of range", problem);
    const Prob &q = plan->probs[problem];
    if (q.d.m != 0) return fail(plan, FDETD_E_ARG, "envelope_gather: problem %d has m = %d (needs m = 0)", problem, q.d.m);
    const size_t eb = elem_bytes(plan->precision);
    if (n < 0 || !aligned(pond, eb / 2) || (n > 0 && (!aligned(samples, 8) || !aligned(out, 8))))
        return fail(plan, FDETD_E_ARG, "envelope_gather: bad arguments");
    if (n == 0) return FDETD_OK;
    EnvGatherArgs G;
    std::memset(&G, 0, sizeof G);
    G.n = n;
    G.samples = samples;
    G.out = out;
    G.pond = pond;
    G.prim = (double *)q.buf[0];  // 2 planes of doubles fit the stage vector (a, a~) in either precision
    G.nz = q.d.nz;
    G.nr = q.d.nr;
    G.nd = q.nd;
    G.dz = q.d.dz;
    G.dr = q.d.dr;
    for (int j = 0; j < q.nd; ++j) G.s[j] = q.s[j];
    HIPCHK(plan, launch_envelope_gather(prec_code(plan->precision), G, plan->stream));
    return FDETD_OK;
}

int envelope_absorber(fdetd_plan_t plan, int32_t problem, int32_t lz, int32_t lr, double sigma_max, double power)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "envelope_absorber: NULL plan");
    if (plan->kind != FDETD_ENVELOPE) return fail(plan, FDETD_E_ARG, "envelope_absorber: plan is not an envelope plan");
    const int np = (int)plan->probs.size();
    if (problem < -1 || problem >= np || lz < 0 || lr < 0 || !(sigma_max >= 0.0) || !std::isfinite(sigma_max) ||
        !(power >= 0.0) || !std::isfinite(power))
        return fail(plan, FDETD_E_ARG, "envelope_absorber: bad arguments");
    const int p0 = problem < 0 ? 0 : problem, p1 = problem < 0 ? np : problem + 1;
    const bool on = sigma_max > 0.0 && (lz > 0 || lr > 0);
    for (int p = p0; p < p1; ++p) {
        const Prob &q = plan->probs[p];
        if (2 * lz > q.d.nz || lr > q.d.nr)
            return fail(plan, FDETD_E_ARG, "envelope_absorber: problem %d: layers wider than the grid", p);
        // the central exponential carries chi + sigma^2: its spectral radius grows by at most sigma_max per
        // layer that can overlap (z and rho in the corners)
        const double smax = sigma_max * ((lz > 0) + (lr > 0));
        if (on && q.rho_hat > 0.0 && q.d.dt * (q.rho_hat + smax) * 1.02 >= taylor_stability_bound(q.d.taylor_order))
            return fail(plan, FDETD_E_UNSTABLE, "envelope_absorber: problem %d: dt (rho + sigma_max) = %.4f exceeds the "
                        "Taylor order-%d bound %.4f / 1.02", p, q.d.dt * (q.rho_hat + smax), q.d.taylor_order,
                        taylor_stability_bound(q.d.taylor_order));
    }
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    const size_t eb = elem_bytes(plan->precision);
    for (int p = p0; p < p1; ++p) {
        Prob &q = plan->probs[p];
        const int nz = q.d.nz, nr = q.d.nr;
        // layer functions: sigma_max d^power, d = depth into the layer / width, 1 on the outermost cell
        std::vector<double> hz(nz, 0.0), hr(nr, 0.0);
        if (on) {
            for (int i = 0; i < lz; ++i) {
                const double v = sigma_max * std::pow((double)(lz - i) / lz, power);
                hz[i] = v;
                hz[nz - 1 - i] = v;
            }
            for (int k = 0; k < lr; ++k) hr[nr - 1 - k] = sigma_max * std::pow((double)(lr - k) / lr, power);
        }
        HIPCHK(plan, hipMemcpy(q.sz, hz.data(), nz * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(plan, hipMemcpy(q.sr, hr.data(), nr * sizeof(double), hipMemcpyHostToDevice));
        // bytes of the two damping passes over the layer cells: (a, a~) read and written, FP32C also lo
        const int64_t old_cells = (int64_t)q.lr * nz + (int64_t)(nr - q.lr) * 2 * q.lz;
        q.lz = on ? lz : 0;
        q.lr = on ? lr : 0;
        const int64_t cells = (int64_t)q.lr * nz + (int64_t)(nr - q.lr) * 2 * q.lz;
        const int64_t per_cell = 2 * 2 * 2 * ((int64_t)eb + (plan->precision == FDETD_FP32C ? 8 : 0));
        plan->info.bytes_per_step += (cells - old_cells) * per_cell;
    }
    if (plan->gexec) {  // the next call captures anew, with or without the damping launches
        (void)hipGraphExecDestroy(plan->gexec);
        plan->gexec = nullptr;
        plan->gkey.clear();
    }
    return FDETD_OK;
}

int fdetd_query(fdetd_plan_t plan, fdetd_plan_info *info)
{
    if (!plan || !info) return fail(plan, FDETD_E_ARG, "fdetd_query: NULL argument");
    *info = plan->info;
    info->profiled_launches = 0;
    info->profiled_ms = 0.0;
    info->profiled_bytes = 0.0;
    if (plan->ev_used) {
        HIPCHK(plan, hipStreamSynchronize(plan->stream));
        for (size_t e = 0; e + 1 < plan->ev_used; e += 2) {
            float ms = 0.f;
            HIPCHK(plan, hipEventElapsedTime(&ms, plan->ev_pool[e], plan->ev_pool[e + 1]));
            info->profiled_ms += ms;
            info->profiled_bytes += plan->ev_bytes[e / 2];
            info->profiled_launches += 1;
        }
        plan->ev_used = 0;
        plan->ev_bytes.clear();
    }
    return FDETD_OK;
}

}  // extern "C"

namespace {
struct StepCtx {
    void *const *psi;
    const void *const *j;
    int64_t stride;
    int n_steps;
};
struct EnvCtx {
    void *const *a;
    void *const *at;
    const void *const *chi;
    int64_t stride;
    int n_steps;
};

int step_body(fdetd_plan_t P, void *vctx)
{
    StepCtx &c = *(StepCtx *)vctx;
    const size_t eb = elem_bytes(P->precision);
    std::vector<const void *> js(P->probs.size());
    int rc = fork_lanes(P);
    for (int s = 0; s < c.n_steps && !rc; ++s) {
        for (size_t p = 0; p < P->probs.size() && c.j; ++p)
            js[p] = (const char *)c.j[p] + (size_t)(c.stride * s) * cur_planes(P) * P->probs[p].cells * eb;
        for (size_t b = 0; b < P->batches.size() && !rc; ++b)
            rc = enqueue_maxwell_batch(P, P->batches[b], c.psi, c.j ? js.data() : nullptr, s == c.n_steps - 1,
                                       lane_stream(P, P->batches[b]));
    }
    const int rj = join_lanes(P);  // also after an error, so that a capture ends with every stream joined
    return rc ? rc : rj;
}

// The generated current of step `step` for the problems of batch b (fdetd_step_graph), on stream s: the
// generator kernel overwrites their blocks (the bunch recipe, or zeros), then the samples' J_z is added.
int enqueue_jgen(fdetd_plan_t P, const Batch &b, const fdetd_jgen &g, int64_t step, void *const *jw, hipStream_t s)
{
    const int prec = prec_code(P->precision);
    JgenArgs J;
    std::memset(&J, 0, sizeof J);
    J.probs = P->ddesc + b.d0;
    J.nprob = b.count;
    J.mode = g.kind == FDETD_JGEN_BUNCH ? 1 : 0;
    J.step = step;
    J.seed = g.seed;
    J.nb = g.nb;
    J.sigz = g.sigz;
    J.sigr = g.sigr;
    J.z0f = g.z0_frac;
    J.vb = g.vb;
    J.amp = g.noise * g.nb;
    size_t max_cells = 0;
    for (int t = 0; t < b.count; ++t) {
        J.pidx[t] = b.members[t];
        J.j[t] = jw[b.members[t]];
        max_cells = std::max(max_cells, P->probs[b.members[t]].cells);
    }
    HIPCHK(P, launch_jgen(prec, J, max_cells, s));
    if (g.kind == FDETD_JGEN_SAMPLES && g.n > 0) {
        DepositArgs A;
        std::memset(&A, 0, sizeof A);
        A.probs = P->ddesc + b.d0;
        A.nprob = b.count;
        A.n = g.n;
        A.samples = g.samples;
        A.vz = g.vz;
        A.eps = g.eps;
        A.shift = g.vz * ((step + 0.5) * b.dt);  // positions at the step's midpoint
        for (int t = 0; t < b.count; ++t) A.j[t] = jw[b.members[t]];
        HIPCHK(P, launch_deposit_jz(prec, A, s));
    }
    return FDETD_OK;
}

struct GraphCtx {
    void *const *psi;
    const fdetd_jgen *g;
    void *const *jw;
    int n_steps;
};

int graph_body(fdetd_plan_t P, void *vctx)
{
    GraphCtx &c = *(GraphCtx *)vctx;
    int rc = fork_lanes(P);
    for (int s = 0; s < c.n_steps && !rc; ++s)
        for (size_t b = 0; b < P->batches.size() && !rc; ++b) {
            const hipStream_t st = lane_stream(P, P->batches[b]);
            if (c.g) rc = enqueue_jgen(P, P->batches[b], *c.g, c.g->step0 + s, c.jw, st);
            if (!rc)
                rc = enqueue_maxwell_batch(P, P->batches[b], c.psi, c.g ? (const void *const *)c.jw : nullptr,
                                           s == c.n_steps - 1, st);
        }
    const int rj = join_lanes(P);
    return rc ? rc : rj;
}

int env_body(fdetd_plan_t P, void *vctx)
{
    EnvCtx &c = *(EnvCtx *)vctx;
    const size_t rb = elem_bytes(P->precision) / 2;
    std::vector<const void *> chis(P->probs.size());
    int rc = fork_lanes(P);
    for (int s = 0; s < c.n_steps && !rc; ++s) {
        for (size_t p = 0; p < P->probs.size(); ++p)
            chis[p] = (const char *)c.chi[p] + (size_t)(c.stride * s) * P->probs[p].cells * rb;
        for (size_t b = 0; b < P->batches.size() && !rc; ++b)
            rc = enqueue_envelope_batch(P, P->batches[b], c.a, c.at, chis.data(), lane_stream(P, P->batches[b]));
    }
    const int rj = join_lanes(P);
    return rc ? rc : rj;
}
}  // namespace

// Replay a captured graph when the call repeats the previous one exactly; otherwise capture anew.
namespace {
int run_maybe_graph(fdetd_plan_t P, const std::vector<const void *> &key, int (*body)(fdetd_plan_t, void *),
                           void *ctx)
{
    if (!(P->flags & FDETD_PLAN_USE_GRAPH)) return body(P, ctx);
    if (!(P->gexec && key == P->gkey)) {
        if (P->gexec) {
            (void)hipGraphExecDestroy(P->gexec);
            P->gexec = nullptr;
        }
        HIPCHK(P, hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
        int rc = body(P, ctx);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(P->stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(P, FDETD_E_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            P->gexec = nullptr;
            return fail(P, FDETD_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        P->gkey = key;
    }
    HIPCHK(P, hipGraphLaunch(P->gexec, P->stream));
    return FDETD_OK;
}
}  // namespace

extern "C" {


int fdetd_step(fdetd_plan_t plan, void *const *psi, const void *const *j_half, int64_t j_step_blocks,
               int32_t n_steps)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_step: NULL plan");
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_step: plan is not a Maxwell plan");
    if (!psi || n_steps < 0 || j_step_blocks < 0) return fail(plan, FDETD_E_ARG, "fdetd_step: bad arguments");
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        const size_t eb = elem_bytes(plan->precision);
        if (!aligned(psi[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_step: psi[%zu] NULL or not %zu-byte aligned", p, eb);
        if (j_half && !aligned(j_half[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_step: j_half[%zu] NULL or not %zu-byte aligned", p, eb);
    }
    if (n_steps == 0) return FDETD_OK;
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        Prob &q = plan->probs[p];
        if (plan->precision == FDETD_FP32C && q.last_state != psi[p] && !plan->adopt_next) {
            int rc = zero_device(plan, q.lo, 6 * q.cells * 8);
            if (rc) return rc;
        }
        q.last_state = psi[p];
    }
    plan->adopt_next = false;
    StepCtx c{psi, j_half, j_step_blocks, n_steps};
    std::vector<const void *> key;
    key.push_back((const void *)(intptr_t)n_steps);
    key.push_back((const void *)(intptr_t)j_step_blocks);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        key.push_back(psi[p]);
        key.push_back(j_half ? j_half[p] : nullptr);
    }
    return run_maybe_graph(plan, key, step_body, &c);
}

int fdetd_step_graph(fdetd_plan_t plan, void *const *psi, const fdetd_jgen *jgen, void *const *j_work, int32_t n_steps)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_step_graph: NULL plan");
    if (plan->kind != FDETD_MAXWELL) return fail(plan, FDETD_E_ARG, "fdetd_step_graph: plan is not a Maxwell plan");
    if (plan->flags & FDETD_PLAN_CURRENT_CORRECTION)
        return fail(plan, FDETD_E_ARG, "fdetd_step_graph: the generated blocks carry no rho_xy for the current correction");
    if (!psi || n_steps < 0 || (jgen && !j_work)) return fail(plan, FDETD_E_ARG, "fdetd_step_graph: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        if (!aligned(psi[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: psi[%zu] NULL or not %zu-byte aligned", p, eb);
        if (jgen && !aligned(j_work[p], eb))
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: j_work[%zu] NULL or not %zu-byte aligned", p, eb);
    }
    if (jgen) {
        const fdetd_jgen &g = *jgen;
        if (g.kind != FDETD_JGEN_BUNCH && g.kind != FDETD_JGEN_SAMPLES)
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: unknown generator kind %d", g.kind);
        if (g.step0 < 0 || g.step0 > ((int64_t)1 << 52))
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: step0 out of range");
        if (g.kind == FDETD_JGEN_BUNCH &&
            (!(g.nb > 0) || !(g.sigz > 0) || !(g.sigr > 0) || !(g.noise >= 0) ||
             !std::isfinite(g.nb + g.sigz + g.sigr + g.noise + g.z0_frac + g.vb)))
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: bunch needs finite nb, sigz, sigr > 0, noise >= 0");
        if (g.kind == FDETD_JGEN_SAMPLES &&
            (g.n < 0 || (g.n > 0 && !aligned(g.samples, 8)) || !(g.eps >= 0.0 && g.eps <= 1.0) || !std::isfinite(g.vz)))
            return fail(plan, FDETD_E_ARG, "fdetd_step_graph: samples need n >= 0, aligned samples, eps in [0, 1], finite vz");
    }
    if (n_steps == 0) return FDETD_OK;
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        Prob &q = plan->probs[p];
        if (plan->precision == FDETD_FP32C && q.last_state != psi[p] && !plan->adopt_next) {
            int rc = zero_device(plan, q.lo, 6 * q.cells * 8);
            if (rc) return rc;
        }
        q.last_state = psi[p];
    }
    plan->adopt_next = false;
    GraphCtx c{psi, jgen, j_work, n_steps};
    // the key of a captured step_graph loop starts with a marker no fdetd_step key has (n_steps >= 1 there)
    std::vector<const void *> key;
    key.push_back((const void *)(intptr_t)-1);
    key.push_back((const void *)(intptr_t)n_steps);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        key.push_back(psi[p]);
        key.push_back(jgen ? j_work[p] : nullptr);
    }
    if (jgen) {
        const fdetd_jgen &g = *jgen;
        auto bits = [](double x) {
            uint64_t u;
            std::memcpy(&u, &x, sizeof u);
            return (const void *)(uintptr_t)u;
        };
        for (const void *v : {(const void *)(intptr_t)g.kind, (const void *)(intptr_t)g.step0, (const void *)(uintptr_t)g.seed,
                              bits(g.nb), bits(g.sigz), bits(g.sigr), bits(g.z0_frac), bits(g.vb), bits(g.noise),
                              (const void *)g.samples, (const void *)(intptr_t)g.n, bits(g.vz), bits(g.eps)})
            key.push_back(v);
    }
    return run_maybe_graph(plan, key, graph_body, &c);
}

int envelope_step(fdetd_plan_t plan, void *const *a, void *const *a_tilde, const void *const *chi_half,
                  int64_t chi_step_planes, int32_t n_steps)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "envelope_step: NULL plan");
    if (plan->kind != FDETD_ENVELOPE) return fail(plan, FDETD_E_ARG, "envelope_step: plan is not an envelope plan");
    if (!a || !a_tilde || !chi_half || n_steps < 0 || chi_step_planes < 0)
        return fail(plan, FDETD_E_ARG, "envelope_step: bad arguments");
    const size_t eb = elem_bytes(plan->precision);
    for (size_t p = 0; p < plan->probs.size(); ++p)
        if (!aligned(a[p], eb) || !aligned(a_tilde[p], eb) || !aligned(chi_half[p], eb / 2))
            return fail(plan, FDETD_E_ARG, "envelope_step: pointer of problem %zu NULL or misaligned", p);
    if (n_steps == 0) return FDETD_OK;
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        Prob &q = plan->probs[p];
        if (plan->precision == FDETD_FP32C && q.last_state != a[p] && !plan->adopt_next) {
            int rc = zero_device(plan, q.lo, 2 * q.cells * 8);
            if (rc) return rc;
        }
        q.last_state = a[p];
    }
    plan->adopt_next = false;
    EnvCtx c{a, a_tilde, chi_half, chi_step_planes, n_steps};
    std::vector<const void *> key;
    key.push_back((const void *)(intptr_t)n_steps);
    key.push_back((const void *)(intptr_t)chi_step_planes);
    for (size_t p = 0; p < plan->probs.size(); ++p) {
        key.push_back(a[p]);
        key.push_back(a_tilde[p]);
        key.push_back(chi_half[p]);
    }
    return run_maybe_graph(plan, key, env_body, &c);
}

int fdetd_export_state(fdetd_plan_t plan, void *host_blob, size_t *bytes)
{
    if (!plan || !bytes) return fail(plan, FDETD_E_ARG, "fdetd_export_state: NULL argument");
    const int np = planes(plan->kind);
    size_t need = 0;
    if (plan->precision == FDETD_FP32C)
        for (auto &q : plan->probs) need += np * q.cells * 8;
    if (!host_blob || *bytes < need) {
        *bytes = need;
        return host_blob ? fail(plan, FDETD_E_ARG, "fdetd_export_state: buffer too small") : FDETD_OK;
    }
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    size_t off = 0;
    for (auto &q : plan->probs) {
        if (plan->precision != FDETD_FP32C) break;
        HIPCHK(plan, hipMemcpy((char *)host_blob + off, q.lo, np * q.cells * 8, hipMemcpyDeviceToHost));
        off += np * q.cells * 8;
    }
    *bytes = need;
    return FDETD_OK;
}

int fdetd_import_state(fdetd_plan_t plan, const void *host_blob, size_t bytes)
{
    if (!plan) return fail(nullptr, FDETD_E_ARG, "fdetd_import_state: NULL plan");
    const int np = planes(plan->kind);
    size_t need = 0;
    if (plan->precision == FDETD_FP32C)
        for (auto &q : plan->probs) need += np * q.cells * 8;
    if (bytes != need || (need && !host_blob))
        return fail(plan, FDETD_E_ARG, "fdetd_import_state: expected %zu bytes, got %zu", need, bytes);
    HIPCHK(plan, hipStreamSynchronize(plan->stream));
    size_t off = 0;
    for (auto &q : plan->probs) {
        if (plan->precision != FDETD_FP32C) break;
        HIPCHK(plan, hipMemcpy(q.lo, (const char *)host_blob + off, np * q.cells * 8, hipMemcpyHostToDevice));
        off += np * q.cells * 8;
    }
    plan->adopt_next = true;
    return FDETD_OK;
}

}  // extern "C"

namespace fdetd {

// Sizes, tiling and coefficient tables of one problem's descriptor (pointers and tile offsets left zero):
// strips of the wavefront width, segments of seg rows below the FP32C near-axis rows (rows 0 .. 2 N_D - 1
// in segments of 8 rows and strips of the near-axis width), the staggered, half-shift, centred and axis
// weights of section 2.3 / 2.4 scaled by the cell sizes.
void describe_problem(const fdetd_problem_desc &d, int precision, int seg, ProbDesc &D)
{
    std::memset(&D, 0, sizeof D);
    const int nd = d.fd_order / 2;
    const int cpw = march_columns_per_wave(prec_code(precision));
    D.nz = d.nz;
    D.nr = d.nr;
    D.m = d.m;
    D.taylor = d.taylor_order;
    D.nd = nd;
    D.nstrip = (d.nz + cpw - 1) / cpw;
    if (precision == FDETD_FP32C) {
        D.ax_rows = std::min(d.nr, axis_band_rows(nd));
        if (D.ax_rows > 0) {
            D.seg_ax = std::min(axis_segment_rows(), D.ax_rows);
            D.nseg_ax = (D.ax_rows + D.seg_ax - 1) / D.seg_ax;
            D.nstrip_ax = (d.nz + axis_columns(nd) - 1) / axis_columns(nd);
        }
    }
    D.seg_rows = seg;
    D.nseg = (d.nr - D.ax_rows + seg - 1) / seg;
    D.plane = (size_t)d.nz * d.nr;
    D.dr = d.dr;
    D.dz = d.dz;
    D.dt = d.dt;
    D.pS = parity_mS(d.m);
    D.k0 = d.k0;
    double a[kMaxND], sh[kMaxND], c[kMaxND], d1[kMaxND], d2[kMaxND + 1];
    make_coefficients(COEF_STAGGERED, nd, a);
    make_coefficients(COEF_HALFSHIFT, nd, sh);
    make_coefficients(COEF_AXIS, nd, c);
    make_coefficients(COEF_CENTRED_D1, nd, d1);
    make_coefficients(COEF_CENTRED_D2, nd, d2);
    for (int k = 0; k < nd; ++k) {
        D.az[k] = a[k] / d.dz;
        D.ar[k] = a[k] / d.dr;
        D.cax[k] = c[k];
        D.sh[k] = sh[k];
        D.dzc[k] = d1[k] / d.dz;
        D.drc[k] = d1[k] / d.dr;
    }
    for (int k = 0; k <= nd; ++k) {
        D.bz[k] = d2[k] / (d.dz * d.dz);
        D.br[k] = d2[k] / (d.dr * d.dr);
    }
    for (int k = 0; k < kMaxND; ++k) {
        D.azf[k] = (float)D.az[k];
        D.arf[k] = (float)D.ar[k];
        D.dzcf[k] = (float)D.dzc[k];
        D.drcf[k] = (float)D.drc[k];
    }
    for (int k = 0; k <= kMaxND; ++k) {
        D.bzf[k] = (float)D.bz[k];
        D.brf[k] = (float)D.br[k];
    }
}

void set_last_error(const char *msg) { g_last_error = msg; }

int default_segment_rows(int precision, const fdetd_problem_desc &d)
{
    const int cpw = march_columns_per_wave(prec_code(precision));
    return default_seg_rows((int64_t)2 * ((d.nz + cpw - 1) / cpw) * d.nr);
}

}  // namespace fdetd
