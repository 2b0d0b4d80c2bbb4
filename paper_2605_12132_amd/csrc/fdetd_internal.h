// Internal declarations shared by the host runtime (fdetd_plan.cpp), the coefficient generator
// (fdetd_coeffs.cpp) and the gfx950 kernels (fdetd_kernels.hip).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime_api.h>

#include "../../include/fdetd.h"

#include <cstddef>
#include <cstdint>

namespace fdetd {

constexpr int kMaxND = 16;  // fd_order <= 32

enum { COEF_STAGGERED = 0, COEF_HALFSHIFT = 1, COEF_CENTRED_D1 = 2, COEF_CENTRED_D2 = 3, COEF_AXIS = 4 };

bool make_coefficients(int which, int nd, double *out);
double taylor_stability_bound(int N);

enum Prec { P64 = 0, P32 = 1 };

// Component order inside a 6-plane Maxwell vector.
enum { ER = 0, ETH = 1, EZ = 2, BR = 3, BTH = 4, BZ = 5 };

// One Horner stage of the Maxwell propagator for one problem:
//   vout = w + coef * H vin,    w = psi + beta * Jbar   (Jbar only in the E slots)
// In the first stage of a step the input is w_N = psi + beta_in * Jbar, formed while loading (vin = psi).
// FP32C: the last stage (vout == psi_hi) adds the increment into the (hi, lo) pair instead of storing w.
struct MaxwellStageArgs {
    const void *vin;
    const void *psi;
    const void *jr, *jt, *jz;  // Jbar planes (jr on the staggered rho grid); all null when no source
    void *vout;
    float *lo;                 // FP32C compensation words of psi (6 planes of float2); null otherwise
    const double *rinv_p;      // 1 / rho_k, k in [0, nr)
    const double *rinv_s;      // 1 / rho_(-),k for k >= 1, 0 at the axis
    double beta_in, beta, coef;
    double dr;
    double pS;                 // +1 / -1: radial extension sign of scalar-like (mS) components
    int nz, nr, m;
    int first, has_src, last_compensated;
    int axis_rows;             // rows k < axis_rows use FP64 arithmetic in the FP32C kernels
    double az[kMaxND];         // a_j / dz
    double ar[kMaxND];         // a_j / dr
    double cax[kMaxND];        // axis extrapolation weights c_k'
};

struct EnvelopeStageArgs {
    const void *vin_a, *vin_t;  // stage input (a, a~)
    const void *psi_a, *psi_t;  // state at t
    const void *chi;            // real plane
    void *out_a, *out_t;
    float *lo_a, *lo_t;         // FP32C compensation (last stage only)
    const double *rinv_p;       // 1 / rho_k
    const double *m2rinv2;      // m^2 / rho_k^2
    double coef, k0, pS;
    int nz, nr, last_compensated, axis_rows;
    double bz[kMaxND + 1];      // centred second-difference weights / dz^2 (b_0 .. b_nd)
    double br[kMaxND + 1];      // ... / dr^2
    double dzc[kMaxND];         // centred first-difference weights / dz
    double drc[kMaxND];         // ... / dr
};

struct AxisArgs {
    void *psi;  // 6 planes
    int nz, nr, m;
    double cax[kMaxND];
};

// ---------------------------------------------------------------------------------------------------
// Row-marching stage kernels (fdetd_march.hip), batched over problems of equal N_D, N and dt.
// ---------------------------------------------------------------------------------------------------
// Near-axis tiles of FP32 storage (FP64 arithmetic): up to N_D = kAxisWholeND each lane holds a whole
// complex value (64 columns per wavefront, like the main tiles); wider stencils need twice the window
// registers and read the storage in lane pairs instead (32 columns per wavefront).
constexpr int kAxisWholeND = 8;
constexpr int kAxisColumns = 32;  // the narrower width; divides every tile width
constexpr int axis_columns(int nd) { return nd <= kAxisWholeND ? 64 : kAxisColumns; }
constexpr int kMaxBatch = 64;  // problems per launch (pointer arrays travel in the kernel arguments)

// Static per-problem facts, uploaded once at plan time.
struct ProbDesc {
    int nz, nr, m, taylor;
    int nd;                                  // stencil half width N_D (launches that mix widths)
    int nstrip;                              // tiling: strips of z columns ...
    int seg_rows, nseg;                      // ... x segments of seg_rows rows from row ax_rows down (main tiles)
    int seg_ax, nseg_ax, ax_rows, nstrip_ax; // FP32C: rows 0 .. ax_rows-1 (= 2 N_D) in segments of seg_ax rows
                                             // and strips of kAxisColumns columns, FP64 arithmetic (near-axis
                                             // tiles); FP64 plans: 0, 0, 0, 0
    int tile_begin, tile_begin_ax;           // first tile of this problem in the main / near-axis launch
    int tile_order;                          // 0: tiles numbered half, segment, strip; 1: segment, half, strip
    size_t plane;                            // nz * nr
    double dr, pS, k0;
    double dz, dt;                           // cell length in z and time step (sample deposition)
    void *buf[2];                            // ping-pong stage vectors
    const void *jbar;                        // staggered J_rho plane
    float *lo;                               // FP32C compensation words
    const double *rinv_p, *rinv_s, *m2rinv2;
    const void *jth;                         // current correction: the corrected J_theta plane the stages read
                                             // instead of the caller's (null without correction)
    const double *sz, *sr;                   // envelope absorbing layer: sigma_z per column, sigma_rho per
                                             // row (all zero without a layer); null for Maxwell problems
    void *pbuf;                              // FP32C increment form: P = H psi of the step (6 planes)
    const void *zero;                        // FP32C increment form: 6 zero planes of at least this size
    double az[kMaxND], ar[kMaxND], cax[kMaxND];          // Maxwell
    double sh[kMaxND];                                   // half-shift weights s_j (current staging)
    double bz[kMaxND + 1], br[kMaxND + 1], dzc[kMaxND], drc[kMaxND];  // envelope
    // the same stencil tables rounded to float, for float arithmetic (its operands are these roundings)
    float azf[kMaxND], arf[kMaxND];
    float bzf[kMaxND + 1], brf[kMaxND + 1], dzcf[kMaxND], drcf[kMaxND];
};

// Descriptor of one problem (sizes, tiling with seg rows per segment, coefficient tables; pointers and
// tile offsets zero), and the default segment length of a single-problem plan.  fdetd_plan.cpp.
void describe_problem(const fdetd_problem_desc &d, int precision, int seg, ProbDesc &D);
int default_segment_rows(int precision, const fdetd_problem_desc &d);
// The message fdetd_last_error(NULL) returns on this thread.
void set_last_error(const char *msg);

// One launch: stage n of every problem in the batch.
struct BatchArgs {
    const ProbDesc *probs;  // device table (the batch's problems are consecutive entries)
    int nprob;
    int ntiles, ntiles_ax;  // main tiles and (FP32 storage) near-axis tiles, FP64 arithmetic, in one launch
    int n, N;               // stage index n (N-1 .. 0) and Taylor order N
    int has_src, compensated;
    // FP32C increment form (Maxwell): the stage vector is the increment d = v - psi, and stage n writes
    // d_n = beta_n Jbar + coef (P + H d_{n+1}) with P = H psi formed once per step (role 1: P = H psi_lo
    // from zero, role 2: P += H psi_hi; role 0: a Horner stage), the last stage TwoSum(psi_hi, lo + d_0)
    int increment, role;
    // the first stage with a current forms the E part of w_N from psi and Jbar as it loads them (no
    // k_form_wn pass before it): the Horner form, not the compensated N = 1 stage
    int fuse_wn;
    int nt_store;  // Maxwell stages store their outputs non-temporal (chosen per batch by the plan's tuning)
    double beta_in, beta, coef;
    const void *psi[kMaxBatch];  // Maxwell psi, or envelope a
    const void *aux[kMaxBatch];  // Maxwell: current of this step (3 planes) or null; envelope: a_tilde
    const void *chi[kMaxBatch];  // envelope: chi of this step
};

template <int ND>
hipError_t march_maxwell_nd(int prec, const BatchArgs &a, hipStream_t s);  // one per N_D, in fdetd_march.hip
template <int ND>
hipError_t march_envelope_nd(int prec, const BatchArgs &a, hipStream_t s);
template <int ND>
hipError_t march_stagger_nd(int prec, const BatchArgs &a, hipStream_t s);
#define FDETD_DECLARE_ND(N)                                                            \
    template <>                                                                        \
    hipError_t march_maxwell_nd<N>(int prec, const BatchArgs &a, hipStream_t s);       \
    template <>                                                                        \
    hipError_t march_envelope_nd<N>(int prec, const BatchArgs &a, hipStream_t s);      \
    template <>                                                                        \
    hipError_t march_stagger_nd<N>(int prec, const BatchArgs &a, hipStream_t s);
FDETD_DECLARE_ND(1) FDETD_DECLARE_ND(2) FDETD_DECLARE_ND(3) FDETD_DECLARE_ND(4) FDETD_DECLARE_ND(5)
FDETD_DECLARE_ND(6) FDETD_DECLARE_ND(7) FDETD_DECLARE_ND(8) FDETD_DECLARE_ND(9) FDETD_DECLARE_ND(10)
FDETD_DECLARE_ND(11) FDETD_DECLARE_ND(12) FDETD_DECLARE_ND(13) FDETD_DECLARE_ND(14) FDETD_DECLARE_ND(15)
FDETD_DECLARE_ND(16)
#undef FDETD_DECLARE_ND
hipError_t launch_maxwell_march(int prec, int nd, const BatchArgs &a, hipStream_t s);   // dispatch on nd
hipError_t launch_envelope_march(int prec, int nd, const BatchArgs &a, hipStream_t s);
hipError_t launch_stagger_march(int prec, int nd, const BatchArgs &a, hipStream_t s);  // aux = the step's currents
int march_columns_per_wave(int prec);  // z columns covered by one wavefront (32 FP64, 64 FP32)
// Launches over batches whose problems differ in N_D (each tile runs its problem's width), in the
// translation units of fdetd_march.hip built with FDETD_ANY_WIDTH = 0 (FP64), 1 (FP32), 2 (FP32 with the
// compensated last stage); dispatched by launch_maxwell_any / launch_stagger_any (fdetd_dispatch.cpp).
hipError_t march_maxwell_any_p64(const BatchArgs &a, hipStream_t s);
hipError_t march_maxwell_any_p32(const BatchArgs &a, hipStream_t s);
hipError_t march_maxwell_any_p32c(const BatchArgs &a, hipStream_t s);
hipError_t march_stagger_any_p64(const BatchArgs &a, hipStream_t s);
hipError_t march_stagger_any_p32(const BatchArgs &a, hipStream_t s);
hipError_t launch_maxwell_any(int prec, const BatchArgs &a, hipStream_t s);
hipError_t launch_stagger_any(int prec, const BatchArgs &a, hipStream_t s);

hipError_t launch_maxwell_stage(int prec, int nd, const MaxwellStageArgs &a, hipStream_t s);
hipError_t launch_envelope_stage(int prec, int nd, const EnvelopeStageArgs &a, hipStream_t s);
hipError_t launch_axis_fix(int prec, int nd, const AxisArgs &a, hipStream_t s);
// The axis rule (section 2.4) on the state of every problem of a batch (a.psi; widths may differ), one
// launch: row 0 of E_rho, B_theta, B_z of problem p = sum_k' c_k' F_k' where the component is constant on
// the axis, else 0.  max_nz: the largest problem's nz.
hipError_t launch_axis_fix_batch(int prec, const BatchArgs &a, int max_nz, hipStream_t s);

// Deposition of point samples into J_z of every problem of a batch (atomic adds in the storage precision).
struct DepositArgs {
    const ProbDesc *probs;  // device table of the batch's problems
    int nprob;
    int64_t n;              // samples
    const double *samples;  // n x 4: z, x, y, q w
    double vz, eps;
    double shift;           // shift of the sample positions along z (charge density; J_z of the in-graph
                            // sample current)
    int rho_xy;             // moving samples: also deposit the planar density differential into plane 3
    void *j[kMaxBatch];     // the problems' current (3 planes; J_z is plane 2), or charge density (1 plane)
};
hipError_t launch_deposit_jz(int prec, const DepositArgs &a, hipStream_t s);
// The current of one step of fdetd_step_graph for the problems of a batch, overwriting their 3-plane
// blocks j[t]: zero (mode 0), or the bunch recipe (mode 1): noise amp (U[-1, 1) of the SplitMix64 stream
// (seed, step, pidx[t]), value ((c nr + k) nz + i) 2 + part; m = 0 keeps real parts) plus, for m = 0,
// -nb exp(-(z - zb)^2 / (2 sigz^2) - rho^2 / (2 sigr^2)) on J_z, zb = z0f nz dz + vb t, t = (step + 1/2) dt.
struct JgenArgs {
    const ProbDesc *probs;
    int nprob, mode;
    int64_t step;
    uint64_t seed;
    double nb, sigz, sigr, z0f, vb, amp;
    int pidx[kMaxBatch];
    void *j[kMaxBatch];
};
hipError_t launch_jgen(int prec, const JgenArgs &a, size_t max_cells, hipStream_t s);
hipError_t launch_deposit_rho(int prec, const DepositArgs &a, hipStream_t s);
hipError_t launch_deposit_current(int prec, const DepositArgs &a, hipStream_t s);  // 8 doubles per sample
// Current correction (section 3.7) of one problem's staged current, three steps:
//   div:   d = rho_xy - D_div^(+,mS) Jbar_rho - (i m / rho) J_theta            -> work (double2 plane)
//   solve: [L_rho^(mS) - m^2/rho^2] phi = d per z column with the plan-time LU factors (no pivoting)
//   apply: Jbar_rho += D_rho^(-,mS) phi (rows >= 1, in place), J_theta~ = J_theta + (i m / rho) phi -> jth
struct CorrectArgs {
    void *jbar;              // staged J_rho (storage precision), corrected in place
    const void *jth_in;      // the caller's J_theta plane
    const void *rho_xy;      // the caller's planar density differential plane
    void *jth_out;           // corrected J_theta (storage precision)
    double2 *work;           // d, then phi (FP64)
    const double *band;      // nr x (2 nd + 1): L below the diagonal, 1/U_kk on it, U above it
    int nz, nr, nd, m, parity;  // parity: m_S sign
    double dr;
    double a[kMaxND];        // staggered first-derivative weights a_j
};
hipError_t launch_correct_div(int prec, const CorrectArgs &a, hipStream_t s);
hipError_t launch_correct_apply(int prec, const CorrectArgs &a, hipStream_t s);
// The banded solves of up to kMaxSolve problems of one N_D.  Each column's rows are split into segments
// solved in parallel from a zero start (the partition method), then a sequential sweep over the segments
// forms the true values at each segment boundary from precomputed responses, and a last parallel pass adds
// each segment's response to its boundary values.  Forward (L) then backward (U) substitution.
constexpr int kMaxSolve = 16;
struct SolveArgs {
    int nprob, nd, smax;  // problems, N_D, most segments of a problem
    struct {
        double2 *work;          // d, then y, then x (in place)
        double2 *wbuf;          // boundary values: [segment][nd][nz]
        const double *band;     // LU factors: rows of 2 nd + 1 (L below the diagonal, 1/U_kk, U above)
        const double *gf, *gb;  // responses [nr][nd] of a segment's rows to a unit value of boundary t
        int nz, nr, seg, nseg;  // rows per segment, segments
    } p[kMaxSolve];
};
hipError_t launch_correct_solve(const SolveArgs &a, hipStream_t s);

// Field interpolation (section 3.3).  Destaggering of one plane to the primary grid: along z (S_z^(+),
// columns outside the grid 0) or along rho (S_rho^(+) with the operand's parity and axis rule).
enum { PASS_Z = 0, PASS_RHO = 1, PASS_COPY = 2, PASS_AXIS = 3 };
struct DestaggerPass {
    const void *src;
    void *dst;
    int op;  // PASS_Z, PASS_RHO: half shift along z / rho; PASS_COPY: copy (2x supersampling);
             // PASS_AXIS: only the axis row, by the axis rule, from rows 1..N_D of dst itself
    int parity, extrapolate;
    int to_stag;    // shifts: 0 staggered -> primary positions (S^(+)); 1 primary -> staggered (S^(-))
    int grow_r;     // rows beyond the box to compute as well
    int set;        // coefficient set (0 or 1) of the problem the planes belong to
    int axis_rule;  // PASS_COPY: the axis row takes the axis rule instead of the stored slot
};
constexpr int kMaxDestaggerPass = 27;
// One launch runs up to kMaxDestaggerPass independent passes (blockIdx.y), over the cells of the box.
struct DestaggerArgs {
    int nz, nr, npass;
    const int *box;  // cells to compute: the samples' footprint (zlo, zhi, klo, khi), clipped to the grid
    int nd[2];
    double s[2][kMaxND];  // half-shift weights s_j
    double c[2][kMaxND];  // axis extrapolation weights c_k'
    DestaggerPass pass[kMaxDestaggerPass];
};
hipError_t launch_destagger(int prec, const DestaggerArgs &a, hipStream_t s);
// The nodes and rows the interpolation shapes of n > 0 samples touch on one grid (zlo, zhi, klo, khi) into
// box: partial boxes of up to max_blocks blocks in part, then one reducing block.
hipError_t launch_gather_box(const double *samples, int64_t n, int nz, int nr, double dz, double dr, int *box,
                             int *part, int max_blocks, hipStream_t s);  // part: 4 max_blocks ints of scratch
constexpr int kMaxGather = 16;  // modes of one grid per gather
struct GatherArgs {
    int64_t n;
    const double *samples;  // n x 4: z, x, y, (unused)
    double *fields;         // n x 6: E_rho, E_theta, E_z, B_rho, B_theta, B_z (overwritten)
    int nprob, nz, nr;
    double dz, dr;
    int m[kMaxGather];
    const void *plane[kMaxGather][6];  // the destaggered components on the primary grid; 2x supersampling:
                                       // the components as stored (the state's planes)
    // 2x supersampling only: plane sets of the doubled grids, component c's set (zs, rs) (1 = staggered
    // position along z, rho) at fine[p] + (4 c + zs + 2 rs) * plane_bytes (the axis rows already hold the
    // axis rule where it applies)
    int ss;                            // bit 0: z doubled, bit 1: rho doubled
    size_t plane_bytes;
    const void *fine[kMaxGather];
};
hipError_t launch_gather(int prec, const GatherArgs &a, hipStream_t s);
// Envelope ponderomotive planes (|a|^2, A~_rho on the staggered rows, A~_z on the staggered columns; real,
// storage precision) at n samples: destaggered on the fly and interpolated, out n x 3 doubles.
struct EnvGatherArgs {
    int64_t n;
    const double *samples;  // n x 4: z, x, y, (unused)
    double *out;
    const void *pond;       // 3 real planes [nr][nz]
    double *prim;           // scratch: A~_rho and A~_z on the primary grid (2 planes of doubles)
    int nz, nr, nd;
    double dz, dr;
    double s[kMaxND];       // half-shift weights s_j
};
hipError_t launch_envelope_gather(int prec, const EnvGatherArgs &a, hipStream_t s);

// Ponderomotive field of an m = 0 envelope problem (section 4.3): 3 real planes |a|^2, A~_rho, A~_z.
hipError_t launch_ponderomotive(int prec, const ProbDesc *d, int nz, int nr, int nd, const void *a, void *out,
                                hipStream_t s);

// Damping exp(-sigma dt/4) of an envelope state (a, a~) on the cells of its absorbing layers: lz columns
// at each z end and lr rows at the outer rho edge.  FP32C: the (hi, lo) pair of each value is scaled in
// FP64 and split again.
struct DampArgs {
    void *a, *at;            // the state planes
    float *lo;               // FP32C compensation words (planes a, a~ of float2), null for FP64
    const double *sz, *sr;   // sigma per column and per row
    int nz, nr, lz, lr;
    double qdt;              // dt / 4
};
hipError_t launch_absorb_damp(int prec, const DampArgs &a, hipStream_t s);
// Per-block partial sums of |x|^2 over n complex values (double2 or float2); nblocks written to partial.
hipError_t launch_norm2(int prec, const void *x, size_t n, double *partial, int nblocks, hipStream_t s);
hipError_t launch_scale(int prec, void *x, size_t n, double alpha, hipStream_t s);
// E part of w_N = psi + beta_in Jbar of every problem of a batch (a.psi, a.aux = the step's currents,
// a.beta_in) into the E planes of each problem's buf[1]; max_cells: the largest problem's nz * nr.
hipError_t launch_form_wn(int prec, const BatchArgs &a, size_t max_cells, hipStream_t s);
// Device-to-device copy of a multiple of 8 bytes by kernel (graph-capture friendly).
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

}  // namespace fdetd
