/*
 * fdetd.h -- C-ABI of the MI355X (gfx950) FDETD library: the finite-difference exponential time-domain
 * field update of a cylindrical (z, rho) particle-in-cell code with azimuthal mode decomposition, and
 * the exponential propagator of the laser-envelope potential (Majorosi, Hafz & Lecz, arXiv 2605.12132).
 *
 * Plain C types and pointers only.  Field, current and susceptibility buffers are DEVICE pointers owned
 * by the caller (any allocator; PyTorch in the provided binding).  All calls enqueue work on the plan's
 * HIP stream and return immediately; results are valid once that stream has synchronised.
 *
 * ---------------------------------------------------------------------------------------------------
 * Storage (all arrays contiguous, each aligned to its element: 16 B FP64 / 8 B FP32C complex,
 * 8 B / 4 B real):
 *   plane          [nr][nz] interleaved complex, z fastest: double2 for FDETD_FP64, float2 for FDETD_FP32C.
 *   Maxwell state  psi: 6 consecutive planes E_rho, E_theta, E_z, B_rho, B_theta, B_z of one azimuthal
 *                  mode m in the complex form F_m = F_{2m} + i F_{2m+1} of the paper's real mode pair
 *                  (section 2.1: the angular derivative acts as i*m).  Yee staggering (Table 1): E_rho,
 *                  B_theta, B_z sit on the staggered radial grid rho_(-),k = k*dr (row 0 is the axis);
 *                  E_theta, E_z, B_rho on rho_k = (k + 1/2) dr; E_z, B_rho, B_theta on the staggered z
 *                  grid z_i - dz/2, the others on z_i = i*dz.
 *                  Row 0 of E_rho, B_theta, B_z is the rho = 0 slot: ignored on input, written on output
 *                  by the boundary rule of section 2.4 (sum_k' c_k' F_k' where the component is constant
 *                  on the axis -- B_z for m = 0, E_rho and B_theta for m = 1 -- and 0 otherwise).
 *   current        j: 3 consecutive planes J_rho, J_theta, J_z at t + dt/2, deposited on the primary
 *                  radial grid (section 2.5 current pre-processing); J_rho and J_theta on z_i, J_z on
 *                  z_i - dz/2.  J_rho is staggered to rho_(-) by the library (S_rho^(-,mA)).
 *   envelope       a, a_tilde: one plane each on the primary grids; chi: [nr][nz] real (double for
 *                  FDETD_FP64, float for FDETD_FP32C), the susceptibility chi_0 at t + dt/2.
 *
 * Errors: every call returns FDETD_OK (0) or a negative code; no exception crosses the ABI.
 * fdetd_last_error() returns a human-readable message for the last failure on that plan
 * (or of the last failed fdetd_plan() or fdetd_step_noalloc() on this thread when called with NULL).
 * ---------------------------------------------------------------------------------------------------
 */
#ifndef FDETD_H
#define FDETD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define FDETD_API __attribute__((visibility("default")))
#else
#define FDETD_API
#endif

#define FDETD_OK          0
#define FDETD_E_ARG      -1  /* bad sizes, order, pointer, alignment or call sequence              */
#define FDETD_E_UNSTABLE -2  /* dt * (estimated spectral radius of H) exceeds the Taylor bound X_N */
#define FDETD_E_NOMEM    -3  /* device allocation failed                                          */
#define FDETD_E_HIP      -4  /* a HIP runtime call failed (message carries hipGetErrorString)       */

#define FDETD_FP64  0        /* everything in double                                                */
#define FDETD_FP32C 1        /* float fields + float compensation word per value (see fdetd_step)   */

#define FDETD_MAXWELL  0
#define FDETD_ENVELOPE 1

/* plan flags */
#define FDETD_PLAN_SKIP_STABILITY 1u  /* do not estimate the spectral radius at plan time           */
#define FDETD_PLAN_USE_GRAPH      2u  /* fdetd_step / envelope_step replay a captured hipGraph        */
#define FDETD_PLAN_PROFILE        4u  /* time every stage kernel with HIP events (not with USE_GRAPH)  */
#define FDETD_PLAN_NO_AUTOTUNE    8u  /* keep the default tiling instead of timing candidates at plan time */
#define FDETD_PLAN_ONE_STREAM    16u  /* enqueue every launch on the plan's stream (no side streams)    */
#define FDETD_PLAN_CURRENT_CORRECTION 32u /* Maxwell: current blocks carry rho_xy; fdetd_step corrects the
                                             staged current every step (section 3.7, see fdetd_step)      */
#define FDETD_PLAN_MIXED_WIDTHS 64u  /* Maxwell: one launch batch for all problems of equal Taylor order and
                                        dt whatever their stencil widths (one launch per stage, two for
                                        FP32C: main and near-axis tiles), instead of one batch per width
                                        on up to four streams; ignored with the current correction        */
#define FDETD_PLAN_PER_WIDTH   128u  /* Maxwell: one launch batch per stencil width.  Without either flag
                                        FP64 plans mix widths and FP32C plans batch per width (the faster
                                        grouping of each on a 64-problem batch of 13 widths); with both,
                                        FDETD_PLAN_PER_WIDTH wins                                          */
#define FDETD_PLAN_INCREMENT_FORM 256u /* FP32C plans (Maxwell and envelope): the Horner stages carry the
                                        increment d_n = v_n - psi instead of v_n (the series of sections
                                        2.1 and 4.2 summed at the size of its terms, not of psi), with
                                        P = H (psi + compensation words) formed once per step by two extra
                                        launches with the stages' own operator; the last stage adds d_0
                                        into the stored (psi, compensation word) pair by TwoSum.  About a
                                        fifth more HBM traffic per step; per-width launch batches.
                                        FDETD_E_ARG for FP64 plans                                         */
#define FDETD_PLAN_SEPARATE_WN 512u  /* Maxwell, steps with a current: form the E part of w_N = psi +
                                        beta_N Jbar (section 2.1) in a pass of its own before the first
                                        Horner stage, instead of in the first stage as it loads psi and
                                        Jbar.
                                        Same results bit for bit; one more launch and ~9 complex values
                                        per cell more traffic per step                                    */

/* Environment variables read when a plan is made (tuning and measurement; none changes a result value):
 *   FDETD_SEG_ROWS      1..4096: rows per marching segment of the main tiles (no autotuning)
 *   FDETD_SEG_AXIS      1..64: rows per segment of the FP32C near-axis tiles (default 16)
 *   FDETD_STORE_POLICY  0 or 1: Maxwell stage outputs stored with the default or non-temporal cache policy
 *                       (otherwise timed at plan time with the segment length)
 *   FDETD_TILE_ORDER    0 or 1: Maxwell tiles numbered half first or segment first (otherwise timed)
 *   FDETD_AUTOTUNE_LOG  set: the tuning's per-candidate times on stderr
 * and one that changes FP32C results, for measuring what the FP64 near-axis band buys:
 *   FDETD_AXIS_ROWS     0..4096: rows next to the axis that FP32C plans compute in FP64 (default 2 N_D) */

typedef struct fdetd_plan_s *fdetd_plan_t;

/* One independent problem: one grid and one azimuthal mode (modes never couple, section 2.1). */
typedef struct {
    int32_t kind;          /* FDETD_MAXWELL or FDETD_ENVELOPE                                      */
    int32_t nz, nr;        /* M_z >= 2*N_D + 1, M_rho >= N_D + 1 (section 2.2)                     */
    int32_t m;             /* azimuthal mode number, 0 <= m <= 64                                 */
    int32_t fd_order;      /* 2*N_D, even, 2..32 (section 2.3 staggered differences)               */
    int32_t taylor_order;  /* N, 1..32: terms of the Taylor sum of each exponential (section 2.5)  */
    double dz, dr, dt;     /* cell sizes and time step, normalised units (c = 1), all > 0          */
    double k0;             /* envelope carrier wavenumber (section 4.1); ignored for Maxwell       */
} fdetd_problem_desc;

typedef struct {
    int32_t n_probs;
    int32_t precision;
    double dt_rho_max;        /* max over problems of dt * estimated spectral radius of H (0: skipped) */
    double stability_margin;  /* min over problems of X_N / (dt * rho_hat) (0: skipped)                */
    int64_t cells;            /* sum over problems of nz * nr                                      */
    int64_t bytes_per_step;   /* algorithmic HBM bytes of one step of all problems                 */
    int64_t scratch_bytes;    /* device memory owned by the plan                                  */
    int64_t launches_per_step;
    /* FDETD_PLAN_PROFILE: stage kernels timed since the previous fdetd_query (query synchronises) */
    int64_t profiled_launches;
    double profiled_ms;          /* sum of their durations                                       */
    double profiled_bytes;       /* sum of their algorithmic HBM bytes                           */
    /* tiling of the first launch batch: rho rows per marching segment of the main launch and of the
     * FP32C near-axis launch (0 without one), and the plan-time autotuning that picked them (0 ms: none) */
    int32_t seg_rows, seg_rows_axis;
    double autotune_ms;
    int32_t streams;  /* streams a step call runs on: 1, or up to 4 when the plan has several launch batches */
    int32_t store_policy;  /* Maxwell stage outputs of the first launch batch: 0 default, 1 non-temporal
                              (timed at plan time with the segment length; FDETD_STORE_POLICY = 0 or 1
                              in the environment fixes it; always 0 for launches that mix widths and for
                              the increment form)                                                   */
    int32_t tile_order;    /* numbering of the Maxwell tiles of the first launch batch: 0 half, segment,
                              strip; 1 segment, half, strip (timed at plan time; FDETD_TILE_ORDER fixes it) */
} fdetd_plan_info;

/* Build a plan for n_probs problems (all FDETD_MAXWELL or all FDETD_ENVELOPE).
 *   probs      host array of n_probs descriptors (copied; caller keeps ownership).
 *   precision  FDETD_FP64 or FDETD_FP32C.
 *   flags      FDETD_PLAN_* bits.
 *   stream     hipStream_t the plan enqueues on (NULL = default stream); the plan is bound to it.
 *   out        receives the plan handle; free it with fdetd_destroy.
 * Generates the coefficient tables in FP64 (section 2.3: staggered, centred and Lagrange weights; section
 * 2.4: axis extrapolation weights), allocates the plan's scratch (ping-pong stage vectors, staggered
 * current, FP32C compensation words) and, unless FDETD_PLAN_SKIP_STABILITY, estimates the spectral radius
 * of each H by power iteration on the GPU and rejects the plan with FDETD_E_UNSTABLE when
 * dt * rho_hat * 1.02 >= X_N (largest x with |T_N(i y)| <= 1 + 1e-9 for all y <= x).  Problems are
 * grouped into launch batches by (fd_order, taylor_order, dt); a plan with several batches also creates
 * up to three side streams (default priority, non-blocking) and runs the batches concurrently: each step
 * call forks them from `stream` with an event and joins them back into it, so the call still orders like
 * work enqueued on `stream` alone (FDETD_PLAN_ONE_STREAM or FDETD_PLAN_PROFILE: no side streams).
 * Synchronises the stream before returning. */
FDETD_API int fdetd_plan(const fdetd_problem_desc *probs, int32_t n_probs, int32_t precision, uint32_t flags,
               void *stream, fdetd_plan_t *out);

/* Advance every Maxwell problem by n_steps midpoint exponential steps (section 2.1, midpoint rule
 * with the factor dt, and the algorithm summary of section 2.5):
 *     psi(t + dt) = T_N(dt H_m) psi(t) - dt * T_N(dt H_m / 2) Jbar(t + dt/2),
 * T_N(X) = sum_{n=0..N} X^n / n!, Jbar = (S_rho^(-,mA) J_rho, J_theta, J_z) (current filters = identity).
 *   psi     n_probs device pointers, each to the 6-plane state of that problem; updated in place.
 *           FDETD_FP32C: float2 planes holding the rounded state; the plan keeps one float compensation
 *           word per real value so that the stored state plus compensation carries ~2x float precision
 *           across steps (export/import with fdetd_export_state / fdetd_import_state).  The
 *           compensation is reset to zero whenever a psi pointer differs from the previous call's,
 *           except on the first call after fdetd_import_state, which adopts the imported words.
 *   j_half  NULL (no current) or n_probs device pointers to 3-plane currents at t + dt/2.
 *   j_step_blocks  distance between the currents of consecutive steps, in blocks of that problem: step s
 *           uses the block starting at j_half[p] + s * j_step_blocks * B * nr_p * nz_p complex values,
 *           B = 3 planes, or 4 with FDETD_PLAN_CURRENT_CORRECTION (1: one block per step stored back to
 *           back; 0: one current for all steps).
 *   FDETD_PLAN_CURRENT_CORRECTION: each block holds a fourth plane, the planar density differential
 *           rho_xy of section 3.7 (primary grid), and after staging every step applies the current
 *           correction of section 3.7:  d = rho_xy - D_div^(+,mS) Jbar_rho - (i m / rho) J_theta,
 *           [L_rho^(mS) - m^2/rho^2] phi = d per z column (L_rho of the centred differences of section
 *           2.3; the plan factors it once, LU without pivoting, FP64), Jbar_rho += D_rho^(-,mS) phi on the
 *           rows k >= 1 and J_theta += (i m / rho) phi (into a plan-owned plane; the caller's current is
 *           only read).  FP64 arithmetic in both precisions.
 *   n_steps >= 0.
 * Enqueue only.  Error (nothing enqueued) on NULL or misaligned pointers or a plan of the wrong kind. */
FDETD_API int fdetd_step(fdetd_plan_t plan, void *const *psi, const void *const *j_half, int64_t j_step_blocks,
               int32_t n_steps);

/* The current of each step of fdetd_step_graph, made inside the time loop (on the GPU, in the captured
 * graph) instead of being held in memory for every step.  Step s of a call is step number step0 + s, at
 * t = (step0 + s + 1/2) dt (the midpoint of section 2.1).  Kinds:
 *   FDETD_JGEN_BUNCH    every problem p (index in the plan) gets J_rho, J_theta, J_z =
 *                       noise * nb * (U_re + i U_im) with U uniform in [-1, 1) from the SplitMix64 stream
 *                       (seed, step, p): value number ((c nr + k) nz + i) 2 + part, c = component, part 0 / 1
 *                       = real / imaginary part, is mix(h + (number + 1) g) with h = mix(mix(mix(seed + g) +
 *                       (step + 1) g) + (p + 1) g), g = 0x9E3779B97F4A7C15, mix the SplitMix64 output function,
 *                       taken as (top 53 bits) 2^-53 * 2 - 1; modes m = 0 keep real parts (section 2.1: the
 *                       imaginary part of m = 0 is discarded); plus on J_z of m = 0 the Gaussian bunch
 *                       -nb exp(-(z_i - dz/2 - zb)^2 / (2 sigz^2) - rho_k^2 / (2 sigr^2)),
 *                       zb = z0_frac nz dz + vb t, rho_k = (k + 1/2) dr.
 *   FDETD_JGEN_SAMPLES  J_rho = J_theta = 0 and J_z deposited from n point samples moving with vz, as
 *                       fdetd_deposit_jz deposits them at the positions z + vz t (samples hold z at t = 0).
 * The generated current replaces the contents of the caller's blocks j_work every step. */
#define FDETD_JGEN_BUNCH   1
#define FDETD_JGEN_SAMPLES 2
typedef struct {
    int32_t kind;            /* FDETD_JGEN_BUNCH or FDETD_JGEN_SAMPLES                            */
    int32_t reserved;        /* 0                                                                 */
    int64_t step0;           /* number of the call's first step (>= 0)                            */
    uint64_t seed;           /* BUNCH: noise stream                                               */
    double nb, sigz, sigr;   /* BUNCH: peak density and widths of the bunch (> 0)                 */
    double z0_frac, vb;      /* BUNCH: bunch centre at t = 0 as a fraction of nz dz, and velocity */
    double noise;            /* BUNCH: noise amplitude relative to nb (>= 0)                      */
    const double *samples;   /* SAMPLES: device array n x 4 (z at t = 0, x, y, q w), 8-byte aligned */
    int64_t n;               /* SAMPLES: number of samples                                        */
    double vz, eps;          /* SAMPLES: velocity along z; radial shape parameter in [0, 1]        */
} fdetd_jgen;

/* n_steps Maxwell steps (as fdetd_step) whose current is made every step by the generator jgen into the
 * caller's blocks j_work[p] (3 planes each, the plan's precision; overwritten every step, and left holding
 * the last step's current).  With FDETD_PLAN_USE_GRAPH the whole loop -- generator, deposition, staging
 * and Horner stages of every step -- is captured once as one hipGraph and replayed by calls that repeat
 * it (same pointers, jgen and n_steps); a replay makes the same steps step0 .. step0 + n_steps - 1 again,
 * and a call with another step0 captures anew.  Without the flag the same launches are enqueued eagerly.
 * FDETD_E_ARG for an envelope plan, a plan with FDETD_PLAN_CURRENT_CORRECTION (its blocks need rho_xy),
 * NULL or misaligned pointers, or bad generator values.  Enqueue only. */
FDETD_API int fdetd_step_graph(fdetd_plan_t plan, void *const *psi, const fdetd_jgen *jgen, void *const *j_work,
                               int32_t n_steps);

/* Advance every envelope problem by n_steps of psi_a(t + dt) = T_N(dt H_a(chi(t + dt/2))) psi_a(t)
 * (section 4.1 exponential solution, section 4.2 discrete operator with L_rho + L_z - m^2/rho^2 and the
 * centred D_z^(C), complex form of the envelope equation with +2 i k0 terms).
 *   a, a_tilde  n_probs device pointers to one plane each; updated in place.
 *   chi_half    n_probs device pointers to real [nr][nz] susceptibility planes; step s uses the plane
 *               at chi_half[p] + s * chi_step_planes * nr_p * nz_p (0: the same plane every step).
 * Enqueue only. */
FDETD_API int envelope_step(fdetd_plan_t plan, void *const *a, void *const *a_tilde, const void *const *chi_half,
                  int64_t chi_step_planes, int32_t n_steps);

/* Deposit the longitudinal current of n point samples (a prescribed particle bunch) into J_z, plane 2
 * of j_half[p], of every problem p of a Maxwell plan, adding to what is there (sections 3.2, 3.5, 3.6):
 *   J_z(z_i - dz/2, rho_k) += q w (F_-(i) - F_+(i)) / dt * R_k * A_m
 * with F_-+(i) the cubic-spline weight of the positions z -+ vz dt/2 on the nodes left of z_i - dz/2 (the
 * integrated shape of section 3.6, signed by the discrete continuity equation), R_k the radial shape of
 * section 3.5 (rho_k^(eps-1) times the spline weight, the part beyond the axis folded back with the mode's
 * m_S type for m = 0, 1 and antisymmetrically for every m > 1, so that a sample on the axis deposits only
 * into m = 0; normalised with the quadrature weights h_0 = 7/8, h_1 = 73/72, h_k = 1) and A_m the
 * deposition form of the angular shape of section 3.2 (1/(2 pi) for m = 0, e^(-i m theta)/pi otherwise,
 * for the mode convention of fdetd_step).  Samples move along z only; a sample whose shape reaches past
 * a z end of a grid is not deposited into it.  F_- - F_+ is non-zero on every node between the two
 * positions, however far apart (a step of more than 3 cells takes a slower path with global atomics).
 *   samples  device array of n x 4 doubles: z, x, y, charge * weight (normalised units), 8-byte aligned.
 *   vz       velocity along z (finite); eps in [0, 1] (0.5 in the paper).
 *   j_half   n_probs device pointers as for fdetd_step (3 planes each, the plan's precision).
 * Enqueue only.  The adds are atomic, so the order of the summation, and the last bits, vary between runs.
 * Blocks of 1024 consecutive samples whose shapes touch at most 4096 cells of a grid sum their adds in an
 * FP64 LDS tile first: samples given in position order (as PIC codes keep them) are much faster. */
FDETD_API int fdetd_deposit_jz(fdetd_plan_t plan, const double *samples, int64_t n, double vz, double eps,
                               void *const *j_half);

/* Deposit the currents of n moving point samples into the current block j_half[p] of every problem of a
 * Maxwell plan, adding to what is there (section 3.6, and section 3.7 for rho_xy).  Positions at the half
 * steps are (z, x, y) +- v dt/2, giving rho+-, theta+-:
 *   J_rho   += q w v_rho   S(z_i - z) R_A(rho_k; rho) A_m(theta)              (plane 0)
 *   J_theta += q w v_theta S(z_i - z) R_A(rho_k; rho) A_m(theta)              (plane 1)
 *   J_z(z_i - dz/2) += q w (F_-(i) - F_+(i)) / dt * (R_S(rho+) A_m(theta+) + R_S(rho-) A_m(theta-)) / 2
 *                                                                             (plane 2, modified Esirkepov)
 *   rho_xy  += q w (S(z_i - z+) + S(z_i - z-)) / 2 * (R_S(rho+) A_m(theta+) - R_S(rho-) A_m(theta-)) / dt
 *                                                   (plane 3, only for plans with FDETD_PLAN_CURRENT_CORRECTION)
 * S(x) = S3(x/dz)/dz; F_-+ and A_m as for fdetd_deposit_jz; R_A / R_S the radial shape of fdetd_deposit_jz
 * folded with the m_A (J_rho, J_theta) / m_S (J_z, rho_xy) type for m = 0, 1, antisymmetrically for m > 1;
 * v_rho = (x v_x + y v_y)/rho and v_theta = (x v_y - y v_x)/rho at the sample, 0 on the axis.  With
 * these, the densities at the end
 * positions satisfy (rho+ - rho-)/dt + D_z^(+) J_z - rho_xy = 0.  A sample whose z shapes reach past a z
 * end is not deposited.  A sample moving more than 3 cells along z in dt (its integrated shape spans
 * more than 8 nodes) is deposited in full with global atomics, outside the LDS tiles.
 *   samples  device array of n x 8 doubles: z, x, y, q w, v_x, v_y, v_z, unused; 8-byte aligned.
 *   eps      in [0, 1].
 *   j_half   n_probs device pointers to current blocks as for fdetd_step (3 planes, 4 with
 *            FDETD_PLAN_CURRENT_CORRECTION), the plan's precision.
 * Enqueue only; atomic adds, summed first in an FP64 LDS tile by blocks of 1024 consecutive samples whose
 * shapes touch at most 1024 cells of a grid (position-ordered samples). */
FDETD_API int fdetd_deposit_current(fdetd_plan_t plan, const double *samples, int64_t n, double eps,
                                    void *const *j_half);

/* Deposit the charge density of n point samples shifted by dz_shift along z into one plane per problem
 * of a Maxwell plan, adding to what is there (sections 3.2, 3.5):
 *   rho(z_i, rho_k) += q w S3(i - (z + dz_shift) / dz) / dz * R_k * A_m
 * with the cubic spline S3 and R_k, A_m as for fdetd_deposit_jz.  With dz_shift = -+ vz dt / 2 the two
 * densities and the current of fdetd_deposit_jz satisfy the discrete continuity equation
 * (rho_+(i) - rho_-(i)) / dt + (J_z(i + 1/2) - J_z(i - 1/2)) / dz = 0.  A sample whose shape reaches past
 * a z end of a grid is not deposited into it.
 *   samples   as for fdetd_deposit_jz; eps in [0, 1].
 *   rho       n_probs device pointers to one complex [nr][nz] plane each, in the plan's precision.
 * Enqueue only; atomic adds as for fdetd_deposit_jz. */
FDETD_API int fdetd_deposit_rho(fdetd_plan_t plan, const double *samples, int64_t n, double dz_shift, double eps,
                                void *const *rho);

/* Fields at n sample positions (section 3.3 field interpolation), for a plan whose problems are modes of
 * one grid (equal nz, nr, dz, dr; at most 16): the components are destaggered to the primary grids,
 *   E_rho = S_rho^(+,mA) E_rho,  E_theta as stored,  E_z = S_z^(+) E_z,  B_rho = S_z^(+) B_rho,
 *   B_theta = S_rho^(+,mA) S_z^(+) B_theta,  B_z = S_rho^(+,mS) B_z
 * (Lagrange half-shifts with the weights s_j, the staggered operand's axis value by the boundary rule,
 * terms beyond the grid 0), then interpolated with cubic shapes in z and rho, the radial shape treated as
 * a Cartesian one over the grid extended below the axis with each component's parity (m_A for the rho and
 * theta components, m_S for the z components), and summed over the modes as Re(F_m e^(i m theta)):
 *   fields[s][c] = sum_m Re( e^(i m theta_s) sum_(i,k) S3(i - z_s/dz) S3(k + 1/2 - rho_s/dr) F_m,c(k, i) ).
 *   psi      n_probs device pointers to the states (as for fdetd_step); read only.
 *   samples  device array of n x 4 doubles (z, x, y, unused), 8-byte aligned.
 *   fields   device array of n x 6 doubles (E_rho, E_theta, E_z, B_rho, B_theta, B_z), overwritten.
 * Uses the plan's stage buffers as scratch (ordered on the plan's stream).  FP32C: destaggers the stored
 * floats (not the compensation words) in FP64 arithmetic and stores the destaggered planes as floats.
 * Enqueue only. */
FDETD_API int fdetd_gather(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n, double *fields);

/* fdetd_gather with the fields' resolution doubled before the shape sum (2x supersampling, section 3.4):
 * supersample bit 0 doubles z, bit 1 doubles rho (0: fdetd_gather itself).  Along a doubled direction a
 * component's nodes are both position sets of the staggered layout, primary and staggered, half a cell
 * apart; the set it is not stored on is filled by a Lagrange half shift of the same order (S^(+) towards
 * primary, S^(-) towards staggered: along z from columns i + j - 1 and i - j, along rho from rows k + j - 1
 * and k - j, the rows below the axis mirrored with the parity, the axis row included), z shifts before rho
 * shifts.  The axis row of a staggered-rho set of a component stored there (E_rho, B_theta, B_z) is the
 * axis rule (extrapolated or 0, as for destaggering).  The cubic shapes are taken in units of the doubled
 * grid, whose rho nodes g drho/2 extend below the axis as parity times node -g:
 *   fields[s][c] = sum_m Re( e^(i m theta_s) sum_(u,g) S3(u - 2 z_s/dz) S3(g - 2 rho_s/dr) F_m,c(u, g) )
 * (a direction not doubled keeps the nodes of fdetd_gather).  Arguments as for fdetd_gather.  The plan
 * allocates 24 planes per problem on the first call (kept until fdetd_destroy; FDETD_E_NOMEM if that
 * fails); FDETD_E_ARG for supersample outside 0..3 or grids of more than 2^29 cells.  Enqueue only. */
FDETD_API int fdetd_gather_supersampled(fdetd_plan_t plan, void *const *psi, const double *samples, int64_t n,
                                        double *fields, int32_t supersample);

/* Ponderomotive field of the envelope model (section 4.3) for the m = 0 problems of an envelope plan:
 *   out[p] plane 0: |a|^2 on the primary grid,
 *          plane 1: A~_rho = -D_rho^(-,mS) |a|^2 on the staggered rho rows k >= 1 (row 0 = 0),
 *          plane 2: A~_z = -D_z^(-) |a|^2 on the staggered z points (z_i - dz/2),
 * with the staggered first-derivative weights of the plan's order, |a|^2 extended evenly below the axis
 * and by 0 beyond the grid.  a: n_probs device pointers to the envelope planes (as for envelope_step);
 * out: n_probs device pointers to 3 real planes of the plan's precision (double / float).  Error
 * FDETD_E_ARG for a Maxwell plan or a problem with m != 0.  Enqueue only. */
FDETD_API int envelope_ponderomotive(fdetd_plan_t plan, const void *const *a, void *const *out);

/* The ponderomotive planes of one m = 0 problem of an envelope plan at n sample positions (section 4.3:
 * |a|^2 and A~ are interpolated at the particles alongside E and B): A~_rho is brought from the staggered
 * rows to the primary ones with S_rho^(+) (odd extension, 0 on the axis), A~_z from the staggered columns
 * with S_z^(+) (0 outside the grid), and the three primary planes are interpolated with the cubic shapes
 * of fdetd_gather over the grid extended below the axis (|a|^2 and A~_z even, A~_rho odd), no angular
 * factor:  out[s][c] = sum_(i,k) S3(i - z_s/dz) S3(k + 1/2 - rho_s/dr) F_c(k, i).
 *   problem  index of an m = 0 problem of the plan.
 *   pond     device pointer to its 3 real planes [nr][nz] (|a|^2, A~_rho, A~_z as envelope_ponderomotive
 *            writes them), the plan's real precision (double for FP64, float for FP32C); read only.
 *   samples  device array of n x 4 doubles (z, x, y, unused), 8-byte aligned.
 *   out      device array of n x 3 doubles, overwritten.
 * FDETD_E_ARG for a Maxwell plan, a problem out of range or with m != 0, or misaligned pointers.
 * Uses the problem's stage buffer as scratch (ordered on the plan's stream).  Enqueue only. */
FDETD_API int envelope_gather(fdetd_plan_t plan, int32_t problem, const void *pond, const double *samples, int64_t n,
                              double *out);

/* Absorbing layers of envelope problems (appendix on the scalar absorbing layer, which the envelope
 * solver of section 4.2 may use): from the next envelope_step on, every step of the problem is
 *     psi_a(t + dt) = exp(-sigma dt/4) T_N(dt H_a(chi~)) exp(-sigma dt/4) psi_a(t),   chi~ = chi + sigma^2,
 * with sigma(z, rho) = sigma_z(z) + sigma_rho(rho) graded as sigma_max d^power: d = (depth of the cell
 * into the layer, in cells) / width, 1 on the outermost cell.  Layers of lz columns at both z ends and lr
 * rows at the outer rho edge; none at the axis.  (The paper defines the layer functions in a companion
 * paper; this grading is the usual PML one.)
 *   problem    index of the problem, or -1 for every problem of the plan.
 *   lz, lr     layer widths in cells: 0 <= 2 lz <= nz, 0 <= lr <= nr (0: no layer on that side).
 *   sigma_max  >= 0, in units of 1/time (0, or lz = lr = 0: remove the layers).
 *   power      >= 0.
 * Error FDETD_E_ARG on an envelope-less plan or bad values; FDETD_E_UNSTABLE when the plan estimated the
 * spectral radius rho_hat and dt (rho_hat + sigma_max per overlapping layer) * 1.02 >= X_N.  Synchronises
 * the plan's stream, then writes the layer tables; a captured graph is captured anew on the next call.
 * FP32C: the damping scales each (value, compensation word) pair in FP64. */
FDETD_API int envelope_absorber(fdetd_plan_t plan, int32_t problem, int32_t lz, int32_t lr, double sigma_max,
                                double power);

/* For callers that cannot allocate device memory -- code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc: fdetd_step for ONE Maxwell problem without a plan, allocating nothing.
 * The step is that of fdetd_step (same kernels, same results bit for bit) with FDETD_PLAN_SKIP_STABILITY
 * and the default tiling.  What a plan would own -- the problem's descriptor, its 1/rho tables, the two
 * stage vectors, the staged current and the FP32C compensation words -- lives in one static device
 * array of 13.7 MB that the library holds on every GPU it runs on until the process ends.
 *   prob     host pointer to the problem (kind FDETD_MAXWELL); nz * nr <= 65536 and nr <= 4096, else
 *            FDETD_E_ARG.
 *   precision, stream: as for fdetd_plan; psi, j_half, j_step_blocks, n_steps: as for fdetd_step with one
 *            problem (single pointers here).
 * FP32C: the compensation words start at zero on every call (they are not carried from one call to the
 * next).  All calls on one GPU share the array: calls that overlap on one GPU (other streams, other host
 * threads) race and give wrong results; calls in order on one stream are safe.  Errors: FDETD_E_ARG (also
 * for sizes beyond the limit), FDETD_E_HIP; the message is fdetd_last_error(NULL).  Enqueue only. */
FDETD_API int fdetd_step_noalloc(const fdetd_problem_desc *prob, int32_t precision, void *stream, void *psi,
                                 const void *j_half, int64_t j_step_blocks, int32_t n_steps);

/* Plan facts (stability estimate, algorithmic bytes per step, scratch size).  Host only. */
FDETD_API int fdetd_query(fdetd_plan_t plan, fdetd_plan_info *info);

/* FP32C compensation words of all problems, problem after problem, 8 bytes per complex value (pass
 * host_blob = NULL to get the size in *bytes).  FDETD_FP64 plans have no state (size 0).  Export
 * synchronises the stream; after import, the next step call keeps the imported words for its pointers. */
FDETD_API int fdetd_export_state(fdetd_plan_t plan, void *host_blob, size_t *bytes);
FDETD_API int fdetd_import_state(fdetd_plan_t plan, const void *host_blob, size_t bytes);

/* Coefficient tables as the library generates them (host only, no GPU needed), FP64:
 *   which 0: staggered first derivative a_1..a_nd      1: Lagrange half shift s_1..s_nd
 *         2: centred first derivative d_1..d_nd       3: centred second derivative b_0..b_nd
 *         4: axis extrapolation c_1..c_nd
 *   out must hold nd + 1 doubles. */
FDETD_API int fdetd_coefficients(int32_t which, int32_t nd, double *out);

/* Largest x with |T_N(i y)| <= 1 + 1e-9 for all 0 <= y <= x (the plan's stability bound). Host only. */
FDETD_API double fdetd_taylor_stability_bound(int32_t taylor_order);

FDETD_API const char *fdetd_last_error(fdetd_plan_t plan);
FDETD_API void fdetd_destroy(fdetd_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif
