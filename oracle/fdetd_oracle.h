/*
 * fdetd_oracle.h -- plain CPU FP64 reference ("oracle") for the FDETD field update and the
 * laser-envelope exponential propagator of Majorosi, Hafz & Lecz, "High-order exponential solver
 * method for particle-in-cell simulations in cylindrical geometry" (arXiv 2605.12132).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call this code:
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no source with the GPU library (its own coefficient formulas, its own ghost rules, its own loops).
 *
 * Storage (identical to what the GPU library documents, so that buffers can be compared):
 *   a "plane" is [nr][nz] double complex, z fastest;
 *   Maxwell state psi = 6 planes in the order E_rho, E_theta, E_z, B_rho, B_theta, B_z;
 *   current j        = 3 planes J_rho, J_theta, J_z, all deposited on the primary rho grid,
 *                      J_rho/J_theta on the primary z grid and J_z on the z grid staggered by -1/2;
 *   envelope         = planes a, a_tilde on the primary grids; chi is [nr][nz] double.
 */
#ifndef FDETD_ORACLE_H
#define FDETD_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nz, nr;          /* M_z, M_rho                                        */
    int32_t m;               /* azimuthal mode number, m >= 0                     */
    int32_t fd_order;        /* 2*N_D, even, 2..32                                */
    int32_t taylor_order;    /* N >= 1                                            */
    int32_t pad_;
    double dz, dr, dt;       /* normalised units, c = 1                           */
    double k0;               /* envelope carrier wavenumber                       */
} oracle_problem;

/* --- finite-difference / interpolation coefficients, order 2*nd (section 2.3, 2.4) --- */
void oracle_coef_staggered(int nd, double *a);     /* a[0..nd-1]: staggered first derivative  */
void oracle_coef_halfshift(int nd, double *s);     /* s[0..nd-1]: Lagrange half-cell shift    */
void oracle_coef_centred_d1(int nd, double *d);    /* d[0..nd-1]: centred first derivative    */
void oracle_coef_centred_d2(int nd, double *b);    /* b[0..nd]: b[0] centre, b[j] pair weight */
void oracle_coef_axis(int nd, double *c);          /* c[0..nd-1]: on-axis extrapolation       */

/* --- single operators on one plane (for pinning the near-axis treatment) ---
 * op: 0 = D_z^(-) (primary z -> staggered z), 1 = D_z^(+) (staggered -> primary),
 *     2 = D_rho^(-) (primary rho -> staggered rho, rows k>=1), 3 = D_rho^(+) (staggered -> primary),
 *     4 = D_div^(-) (primary -> staggered, rows k>=1),      5 = D_div^(+) (staggered -> primary),
 *     6 = S_rho^(-) (primary -> staggered, rows k>=1),
 *     7 = L_rho (primary -> primary), 8 = L_z, 9 = D_z^(C), 10 = axis value of a staggered plane
 *         (written to row 0 of out, all other rows 0).
 * parity: +1 symmetric, -1 antisymmetric extension to rho<0 (for op 3 and 10 also picks the axis rule,
 *         see axis_extrapolate).  axis_extrapolate: 1 = axis value of a staggered operand is the
 *         Lagrange extrapolation sum c_k' f_k', 0 = axis value is zero. */
int oracle_apply_op(const oracle_problem *P, int op, int parity, int axis_extrapolate,
                    const double complex *in, double complex *out);

/* --- Maxwell operator H_m (section 2.5 discrete Ampere/Faraday equations) --- */
int oracle_apply_H(const oracle_problem *P, const double complex *v, double complex *out);
/* J-bar: J_rho staggered by S_rho^(-,mA); J_theta and J_z unchanged (no z filter). */
int oracle_stage_current(const oracle_problem *P, const double complex *j, double complex *jbar);
/* Overwrite the rho = 0 slots of E_rho, B_theta, B_z by the boundary rule (section 2.4). */
int oracle_set_axis(const oracle_problem *P, double complex *psi);
/* n_steps midpoint exponential steps; j may be NULL (no source); step s uses the current block
 * j + s*j_stride (j_stride in complex elements, 0 = same block every step). */
int oracle_step(const oracle_problem *P, double complex *psi, const double complex *j,
                int64_t j_stride, int n_steps);

/* Current correction of section 3.7 on a staged current jbar (3 planes, J_rho staggered) with the planar
 * density differential rho_xy; in place.  oracle_step_corrected: steps whose current blocks hold four
 * planes (J_rho, J_theta, J_z, rho_xy), corrected after staging. */
int oracle_correct_current(const oracle_problem *P, double complex *jbar, const double complex *rho_xy);
int oracle_step_corrected(const oracle_problem *P, double complex *psi, const double complex *j,
                          int64_t j_stride, int n_steps);

/* --- laser envelope (section 4) --- */
int oracle_apply_Ha(const oracle_problem *P, const double complex *a, const double complex *at,
                    const double *chi, double complex *out_a, double complex *out_at);
int oracle_envelope_step(const oracle_problem *P, double complex *a, double complex *at,
                         const double *chi, int n_steps);
/* Ponderomotive field of the envelope model (section 4.3), m = 0: out = 3 real planes |a|^2,
 * A~_rho = -D_rho^(-,mS)|a|^2 (staggered rho), A~_z = -D_z^(-)|a|^2 (staggered z). */
int oracle_ponderomotive(const oracle_problem *P, const double complex *a, double *out);
/* Scalar absorbing layer (appendix on the scalar absorbing layer): layer functions sigma [nr][nz]
 * (polynomial grading over lz columns at both z ends and lr rows at the outer rho edge) and the split
 * step exp(-sigma dt/4) T_N(dt H_a(chi + sigma^2)) exp(-sigma dt/4). */
int oracle_absorber_profile(const oracle_problem *P, int lz, int lr, double sigma_max, double power,
                            double *sigma);
int oracle_envelope_step_absorbing(const oracle_problem *P, double complex *a, double complex *at,
                                   const double *chi, const double *sigma, int n_steps);

/* --- diagnostics (section 5.1) --- */
/* Field energy sum_fields sum_cells w_m r dr dz |F|^2 and its z-centroid (Maxwell state). */
void oracle_energy(const oracle_problem *P, const double complex *psi, double *energy, double *zc);
/* Same for the envelope, integrating |a_tilde - i k0 a|^2. */
void oracle_envelope_energy(const oracle_problem *P, const double complex *a,
                            const double complex *at, double *energy, double *zc);

/* Deposition of point samples (z, x, y, q w per sample; sections 3.2, 3.5, 3.6, with the readings stated in fdetd_oracle.c):
 * the charge density of mode m of the samples shifted by dz_shift along z, and the longitudinal current
 * of samples moving with vz (plane 2 of the 3-plane j).  Both add into their output.  Samples whose z
 * shape reaches past either z end of the grid are not deposited. */
int oracle_deposit_rho(const oracle_problem *P, const double *samples, long n, double dz_shift, double eps,
                       double complex *rho);
int oracle_deposit_jz(const oracle_problem *P, const double *samples, long n, double vz, double eps,
                      double complex *j);

/* Currents of moving samples (section 3.6; 8 doubles per sample: z, x, y, q w, v_x, v_y, v_z, unused) into
 * j (J_rho, J_theta, J_z) and, if not NULL, the planar density differential rho_xy of section 3.7. */
int oracle_deposit_current(const oracle_problem *P, const double *samples, long n, double eps, double complex *j,
                           double complex *rho_xy);

/* Field interpolation (section 3.3): the six components destaggered to the primary grids, and the value
 * of this mode at each sample added into fields (n x 6 doubles). */
int oracle_destagger(const oracle_problem *P, const double complex *psi, double complex *out);
int oracle_interpolate(const oracle_problem *P, const double complex *prim, const double *samples, long n,
                       double *fields);
/* The same with the fields' resolution doubled before the shape sum (section 3.4): ss bit 0 along z,
 * bit 1 along rho (ss = 0: the plain interpolation); the mode's value at each sample is added into fields. */
int oracle_gather_fine(const oracle_problem *P, const double complex *psi, const double *samples, long n, int ss,
                       double *fields);

/* |a|^2, A~_rho, A~_z of an m = 0 envelope ([3][nr][nz] real, as oracle_ponderomotive writes them) at n
 * samples (section 4.3): destaggered to the primary grid and interpolated with cubic shapes; out is n x 3. */
int oracle_envelope_gather(const oracle_problem *P, const double *pond, const double *samples, long n, double *out);

int oracle_num_threads(void);
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
