/*
 * fdetd_oracle.c -- plain, slow, obviously correct CPU FP64 reference of the FDETD field update
 * and of the laser-envelope exponential propagator (arXiv 2605.12132).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product (GPU) path never includes, links or calls it, and the two share no code.
 *
 * The oracle follows the paper's own order of operations:
 *   - every operator is a banded matrix applied row by row (section 2.2, banded-matrix products),
 *     values outside the grid are extended by the radial symmetry rules (section 2.4, Table 1) or
 *     ignored (outside [0, M_z) in z and beyond the last radial node);
 *   - H_m is the discrete Ampere/Faraday system of section 2.5 written in complex modes
 *     (d/dtheta -> i m, the complex form of the real 2x2 rotation of the mode pair);
 *   - a step is the midpoint solution exp(dt H) psi - dt exp(dt H/2) Jbar (section 2.1, with the
 *     factor dt of the midpoint quadrature written out), each exponential being the explicit Taylor
 *     sum sum_{n=0..N} (dt^n / n!) H^n (section 2.5, algorithm summary), summed forward;
 *   - the envelope step is the Taylor sum of exp(dt H_a) (section 4.1/4.2).
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math, no FMA contraction).
 * Parity of this file against the mathematics is pinned by the CPU test suite.
 */
#include "fdetd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define IDX(P, k, i) ((size_t)(k) * (size_t)(P)->nz + (size_t)(i))

enum { ER = 0, ETH = 1, EZ = 2, BR = 3, BTH = 4, BZ = 5 };

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from now on (the CPU baseline times the oracle on one core and on all). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Coefficients.  All are Lagrange-interpolation weights written as closed products.           */
/* ------------------------------------------------------------------------------------------ */

/* Staggered first derivative of order 2*nd (section 2.3, staggered differences D^(+-)):
 * f'(0) ~ sum_j a_j [f((j-1/2)h) - f(-(j-1/2)h)] / h.  Exactness on x^(2p-1), p=1..nd, gives
 * a_j (2j-1) = prod_{i!=j} (2i-1)^2 / ((2i-1)^2 - (2j-1)^2). */
void oracle_coef_staggered(int nd, double *a)
{
    for (int j = 1; j <= nd; ++j) {
        double yj = 2.0 * j - 1.0, prod = 1.0;
        for (int i = 1; i <= nd; ++i) {
            if (i == j) continue;
            double yi = 2.0 * i - 1.0;
            prod *= (yi * yi) / (yi * yi - yj * yj);
        }
        a[j - 1] = prod / yj;
    }
}

/* Lagrange half-cell shift of the same order (section 2.3, S^(+-)):
 * f(0) ~ sum_j s_j [f((j-1/2)h) + f(-(j-1/2)h)],  2 s_j = prod_{i!=j} (2i-1)^2/((2i-1)^2-(2j-1)^2). */
void oracle_coef_halfshift(int nd, double *s)
{
    for (int j = 1; j <= nd; ++j) {
        double yj = 2.0 * j - 1.0, prod = 1.0;
        for (int i = 1; i <= nd; ++i) {
            if (i == j) continue;
            double yi = 2.0 * i - 1.0;
            prod *= (yi * yi) / (yi * yi - yj * yj);
        }
        s[j - 1] = 0.5 * prod;
    }
}

/* Centred (non-staggered) first derivative D^(C) (section 2.3 radial Laplacian, section 4.2):
 * f'(0) ~ sum_j d_j [f(jh) - f(-jh)] / h,  2 j d_j = prod_{i!=j} i^2/(i^2-j^2). */
void oracle_coef_centred_d1(int nd, double *d)
{
    for (int j = 1; j <= nd; ++j) {
        double prod = 1.0;
        for (int i = 1; i <= nd; ++i) {
            if (i == j) continue;
            prod *= ((double)i * i) / ((double)i * i - (double)j * j);
        }
        d[j - 1] = prod / (2.0 * j);
    }
}

/* Centred second derivative D^2 (section 2.3): f''(0) ~ [b_0 f(0) + sum_j b_j (f(jh)+f(-jh))]/h^2,
 * j^2 b_j = prod_{i!=j} i^2/(i^2-j^2), and b_0 = -2 sum_j b_j (constants are annihilated). */
void oracle_coef_centred_d2(int nd, double *b)
{
    double sum = 0.0;
    for (int j = 1; j <= nd; ++j) {
        double prod = 1.0;
        for (int i = 1; i <= nd; ++i) {
            if (i == j) continue;
            prod *= ((double)i * i) / ((double)i * i - (double)j * j);
        }
        b[j] = prod / ((double)j * j);
        sum += b[j];
    }
    b[0] = -2.0 * sum;
}

/* On-axis value of a staggered field that is constant (even) at rho = 0 (section 2.4, axis
 * boundary values): Lagrange extrapolation in rho^2 through the nodes rho = k' drho, k'=1..nd:
 * c_k' = prod_{i!=k'} i^2/(i^2-k'^2).  At nd = 5 this is 5/3, -20/21, 5/14, -5/63, 1/126. */
void oracle_coef_axis(int nd, double *c)
{
    for (int k = 1; k <= nd; ++k) {
        double prod = 1.0;
        for (int i = 1; i <= nd; ++i) {
            if (i == k) continue;
            prod *= ((double)i * i) / ((double)i * i - (double)k * k);
        }
        c[k - 1] = prod;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Grid values with the boundary rules.                                                         */
/* ------------------------------------------------------------------------------------------ */

/* Radial symmetry type of section 2.4: mS is S (even) for even m, A (odd) for odd m;
 * mA is S for even |m-1|, A for odd |m-1|.  Returned as the sign of the extension. */
static int parity_mS(int m) { return (m % 2 == 0) ? +1 : -1; }
static int parity_mA(int m) { return (abs(m - 1) % 2 == 0) ? +1 : -1; }

/* Primary radial grid rho_k = (k+1/2) drho.  A row q<0 is the mirror image of row -1-q (the point
 * -rho_q'), multiplied by the extension sign; rows >= nr and z outside [0, nz) are ignored (0). */
static cplx prim_val(const oracle_problem *P, const cplx *f, int parity, int q, int i)
{
    if (i < 0 || i >= P->nz) return 0.0;
    if (q < 0) {
        int mirror = -1 - q;
        if (mirror >= P->nr) return 0.0;
        return (double)parity * f[IDX(P, mirror, i)];
    }
    if (q >= P->nr) return 0.0;
    return f[IDX(P, q, i)];
}

/* Staggered radial grid rho_(-),q = q drho.  Row 0 is the axis and takes the value 'axis'; a row
 * q<0 mirrors row -q with the extension sign; rows >= nr and z outside [0, nz) are ignored. */
static cplx stag_val(const oracle_problem *P, const cplx *f, int parity, cplx axis, int q, int i)
{
    if (i < 0 || i >= P->nz) return 0.0;
    if (q == 0) return axis;
    if (q < 0) {
        int mirror = -q;
        if (mirror >= P->nr) return 0.0;
        return (double)parity * f[IDX(P, mirror, i)];
    }
    if (q >= P->nr) return 0.0;
    return f[IDX(P, q, i)];
}

/* Axis value of a staggered plane at column i: sum_{k'=1..N_D} c_k' f_k' when the field is constant
 * on the axis, else 0 (section 2.4). */
static cplx axis_value(const oracle_problem *P, const double *c, int nd, const cplx *f, int i,
                       int extrapolate)
{
    if (!extrapolate) return 0.0;
    cplx s = 0.0;
    for (int k = 1; k <= nd; ++k) {
        if (k >= P->nr) break;
        s += c[k - 1] * f[IDX(P, k, i)];
    }
    return s;
}

/* ------------------------------------------------------------------------------------------ */
/* Banded operators (section 2.2 product rule, section 2.3 definitions).                         */
/* ------------------------------------------------------------------------------------------ */

/* D_z^(-): primary z -> staggered z (output at z_i - dz/2). */
static void op_dz_minus(const oracle_problem *P, const double *a, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += a[j - 1] * (prim_val(P, in, +1, k, i + j - 1) - prim_val(P, in, +1, k, i - j));
            out[IDX(P, k, i)] = s / P->dz;
        }
}

/* D_z^(+): staggered z -> primary z. */
static void op_dz_plus(const oracle_problem *P, const double *a, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += a[j - 1] * (prim_val(P, in, +1, k, i + j) - prim_val(P, in, +1, k, i - j + 1));
            out[IDX(P, k, i)] = s / P->dz;
        }
}

/* D_rho^(-): primary rho -> staggered rho, evaluated on the evolved rows k >= 1; the axis row of the
 * result is left 0 (it is not part of the system, section 2.5). */
static void op_dr_minus(const oracle_problem *P, const double *a, int nd, int parity, const cplx *in,
                        cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            if (k >= 1)
                for (int j = 1; j <= nd; ++j)
                    s += a[j - 1] * (prim_val(P, in, parity, k + j - 1, i) - prim_val(P, in, parity, k - j, i));
            out[IDX(P, k, i)] = s / P->dr;
        }
}

/* D_rho^(+): staggered rho -> primary rho; the axis value of the operand is placed into the operator
 * (section 2.4). */
static void op_dr_plus(const oracle_problem *P, const double *a, const double *c, int nd, int parity,
                       int extrapolate, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx ax = axis_value(P, c, nd, in, i, extrapolate);
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += a[j - 1] * (stag_val(P, in, parity, ax, k + j, i) - stag_val(P, in, parity, ax, k - j + 1, i));
            out[IDX(P, k, i)] = s / P->dr;
        }
}

/* D_div^(-) = rho_(-)^-1 D^(-) (rho F): the operand rho*F lives on the primary grid and is extended
 * with the parity given for the operator (section 2.3 staggered divergence).  Rows k >= 1. */
static void op_div_minus(const oracle_problem *P, const double *a, int nd, int parity, const cplx *in,
                         cplx *out)
{
    size_t n = (size_t)P->nr * P->nz;
    cplx *g = malloc(n * sizeof(cplx));
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) g[IDX(P, k, i)] = (k + 0.5) * P->dr * in[IDX(P, k, i)];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            if (k >= 1) {
                for (int j = 1; j <= nd; ++j)
                    s += a[j - 1] * (prim_val(P, g, parity, k + j - 1, i) - prim_val(P, g, parity, k - j, i));
                s = s / P->dr / (k * P->dr);
            }
            out[IDX(P, k, i)] = s;
        }
    free(g);
}

/* D_div^(+) = rho^-1 D^(+) (rho_(-) F): operand rho_(-) F on the staggered grid, zero on the axis
 * (its matrix elements at rho = 0 vanish, section 2.3). */
static void op_div_plus(const oracle_problem *P, const double *a, int nd, int parity, const cplx *in,
                        cplx *out)
{
    size_t n = (size_t)P->nr * P->nz;
    cplx *g = malloc(n * sizeof(cplx));
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) g[IDX(P, k, i)] = (k * P->dr) * in[IDX(P, k, i)];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += a[j - 1] * (stag_val(P, g, parity, 0.0, k + j, i) - stag_val(P, g, parity, 0.0, k - j + 1, i));
            out[IDX(P, k, i)] = s / P->dr / ((k + 0.5) * P->dr);
        }
    free(g);
}

/* S_rho^(-): Lagrange shift primary rho -> staggered rho, rows k >= 1 (section 2.3). */
static void op_shift_minus(const oracle_problem *P, const double *s_, int nd, int parity,
                           const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            if (k >= 1)
                for (int j = 1; j <= nd; ++j)
                    s += s_[j - 1] * (prim_val(P, in, parity, k + j - 1, i) + prim_val(P, in, parity, k - j, i));
            out[IDX(P, k, i)] = s;
        }
}

/* S_rho^(+): Lagrange half-shift staggered rho -> primary rho (section 3.3 destaggering, the
 * counterpart of S^(-) of section 2.3); the operand's axis value is placed in row 0 and its ghosts
 * mirror with the given parity, as for D_rho^(+). */
static void op_shift_plus_rho(const oracle_problem *P, const double *s_, const double *c, int nd, int parity,
                              int extrapolate, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx ax = axis_value(P, c, nd, in, i, extrapolate);
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += s_[j - 1] * (stag_val(P, in, parity, ax, k + j, i) + stag_val(P, in, parity, ax, k - j + 1, i));
            out[IDX(P, k, i)] = s;
        }
}

/* S_z^(+): Lagrange half-shift staggered z -> primary z (section 3.3); terms outside [0, nz) are 0. */
static void op_shift_plus_z(const oracle_problem *P, const double *s_, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += s_[j - 1] * (prim_val(P, in, +1, k, i + j) + prim_val(P, in, +1, k, i - j + 1));
            out[IDX(P, k, i)] = s;
        }
}

/* Radial Laplacian L_rho = D^2 + rho^-1 D^(C) on the primary grid (section 2.3). */
static void op_lap_rho(const oracle_problem *P, const double *b, const double *d, int nd, int parity,
                       const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s2 = b[0] * prim_val(P, in, parity, k, i);
            cplx s1 = 0.0;
            for (int j = 1; j <= nd; ++j) {
                s2 += b[j] * (prim_val(P, in, parity, k + j, i) + prim_val(P, in, parity, k - j, i));
                s1 += d[j - 1] * (prim_val(P, in, parity, k + j, i) - prim_val(P, in, parity, k - j, i));
            }
            double rho = (k + 0.5) * P->dr;
            out[IDX(P, k, i)] = s2 / (P->dr * P->dr) + (s1 / P->dr) / rho;
        }
}

/* L_z = D_z^2 on the primary z grid. */
static void op_lap_z(const oracle_problem *P, const double *b, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = b[0] * prim_val(P, in, +1, k, i);
            for (int j = 1; j <= nd; ++j)
                s += b[j] * (prim_val(P, in, +1, k, i + j) + prim_val(P, in, +1, k, i - j));
            out[IDX(P, k, i)] = s / (P->dz * P->dz);
        }
}

/* D_z^(C): centred first derivative in z. */
static void op_dz_centred(const oracle_problem *P, const double *d, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += d[j - 1] * (prim_val(P, in, +1, k, i + j) - prim_val(P, in, +1, k, i - j));
            out[IDX(P, k, i)] = s / P->dz;
        }
}

static int check_problem(const oracle_problem *P)
{
    if (P->nz < 1 || P->nr < 1) return -1;
    if (P->fd_order < 2 || P->fd_order > 32 || (P->fd_order % 2)) return -1;
    if (P->nr < P->fd_order / 2 + 1) return -1;
    if (P->m < 0) return -1;
    return 0;
}

int oracle_apply_op(const oracle_problem *P, int op, int parity, int axis_extrapolate,
                    const double complex *in, double complex *out)
{
    if (check_problem(P)) return -1;
    int nd = P->fd_order / 2;
    double a[16], s[16], d[16], b[17], c[16];
    oracle_coef_staggered(nd, a);
    oracle_coef_halfshift(nd, s);
    oracle_coef_centred_d1(nd, d);
    oracle_coef_centred_d2(nd, b);
    oracle_coef_axis(nd, c);
    switch (op) {
    case 0: op_dz_minus(P, a, nd, in, out); break;
    case 1: op_dz_plus(P, a, nd, in, out); break;
    case 2: op_dr_minus(P, a, nd, parity, in, out); break;
    case 3: op_dr_plus(P, a, c, nd, parity, axis_extrapolate, in, out); break;
    case 4: op_div_minus(P, a, nd, parity, in, out); break;
    case 5: op_div_plus(P, a, nd, parity, in, out); break;
    case 6: op_shift_minus(P, s, nd, parity, in, out); break;
    case 7: op_lap_rho(P, b, d, nd, parity, in, out); break;
    case 8: op_lap_z(P, b, nd, in, out); break;
    case 9: op_dz_centred(P, d, nd, in, out); break;
    case 11: op_shift_plus_rho(P, s, c, nd, parity, axis_extrapolate, in, out); break;
    case 12: op_shift_plus_z(P, s, nd, in, out); break;
    case 10:
        memset(out, 0, (size_t)P->nr * P->nz * sizeof(cplx));
        for (int i = 0; i < P->nz; ++i) out[IDX(P, 0, i)] = axis_value(P, c, nd, in, i, axis_extrapolate);
        break;
    default: return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Maxwell operator H_m (section 2.5) in complex modes: E_rho, B_theta, B_z on the staggered rho grid, */
/* E_z, B_rho, B_theta on the staggered z grid (Table 1).  Only staggered rows k >= 1 are evolved.     */
/* ------------------------------------------------------------------------------------------ */

int oracle_apply_H(const oracle_problem *P, const double complex *v, double complex *out)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2, m = P->m;
    const size_t n = (size_t)P->nr * P->nz;
    double a[16], c[16];
    oracle_coef_staggered(nd, a);
    oracle_coef_axis(nd, c);
    const int pS = parity_mS(m);
    const cplx *Er = v + ER * n, *Eth = v + ETH * n, *Ez = v + EZ * n;
    const cplx *Br = v + BR * n, *Bth = v + BTH * n, *Bz = v + BZ * n;
    cplx *t = malloc(n * sizeof(cplx));
    cplx *o;

    /* dE_rho = -D_z^(+) B_theta + (i m / rho_(-)) B_z            (rows k >= 1) */
    o = out + ER * n;
    op_dz_plus(P, a, nd, Bth, t);
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i)
            o[IDX(P, k, i)] = (k == 0) ? 0.0 : -t[IDX(P, k, i)] + (I * m / (k * P->dr)) * Bz[IDX(P, k, i)];

    /* dE_theta = D_z^(+) B_rho - D_rho^(+,mS) B_z   (B_z axis value extrapolated iff m = 0) */
    o = out + ETH * n;
    op_dz_plus(P, a, nd, Br, o);
    op_dr_plus(P, a, c, nd, pS, m == 0, Bz, t);
    for (size_t q = 0; q < n; ++q) o[q] -= t[q];

    /* dE_z = -(i m / rho) B_rho + D_div^(+,mS) B_theta */
    o = out + EZ * n;
    op_div_plus(P, a, nd, pS, Bth, o);
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i)
            o[IDX(P, k, i)] += -(I * m / ((k + 0.5) * P->dr)) * Br[IDX(P, k, i)];

    /* dB_rho = D_z^(-) E_theta - (i m / rho) E_z */
    o = out + BR * n;
    op_dz_minus(P, a, nd, Eth, o);
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i)
            o[IDX(P, k, i)] += -(I * m / ((k + 0.5) * P->dr)) * Ez[IDX(P, k, i)];

    /* dB_theta = -D_z^(-) E_rho + D_rho^(-,mS) E_z                (rows k >= 1) */
    o = out + BTH * n;
    op_dz_minus(P, a, nd, Er, t);
    op_dr_minus(P, a, nd, pS, Ez, o);
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i)
            o[IDX(P, k, i)] = (k == 0) ? 0.0 : o[IDX(P, k, i)] - t[IDX(P, k, i)];

    /* dB_z = (i m / rho_(-)) E_rho - D_div^(-,mS) E_theta         (rows k >= 1) */
    o = out + BZ * n;
    op_div_minus(P, a, nd, pS, Eth, o);
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i)
            o[IDX(P, k, i)] = (k == 0) ? 0.0 : (I * m / (k * P->dr)) * Er[IDX(P, k, i)] - o[IDX(P, k, i)];

    free(t);
    /* the rho = 0 slots of the result follow the boundary rule */
    return oracle_set_axis(P, out);
}

int oracle_set_axis(const oracle_problem *P, double complex *psi)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2, m = P->m;
    const size_t n = (size_t)P->nr * P->nz;
    double c[16];
    oracle_coef_axis(nd, c);
    /* E_rho and B_theta are polar-like (mA): constant on the axis only for m = 1.
     * B_z is scalar-like (mS): constant on the axis only for m = 0.  Otherwise zero. */
    for (int i = 0; i < P->nz; ++i) {
        cplx er = axis_value(P, c, nd, psi + ER * n, i, m == 1);
        cplx bt = axis_value(P, c, nd, psi + BTH * n, i, m == 1);
        cplx bz = axis_value(P, c, nd, psi + BZ * n, i, m == 0);
        psi[ER * n + IDX(P, 0, i)] = er;
        psi[BTH * n + IDX(P, 0, i)] = bt;
        psi[BZ * n + IDX(P, 0, i)] = bz;
    }
    return 0;
}

/* Jbar_rho = S_rho^(-,mA) J_rho, Jbar_theta = J_theta, Jbar_z = J_z (section 2.5 current
 * pre-processing with the z filters taken as the identity). */
int oracle_stage_current(const oracle_problem *P, const double complex *j, double complex *jbar)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2;
    const size_t n = (size_t)P->nr * P->nz;
    double s[16];
    oracle_coef_halfshift(nd, s);
    op_shift_minus(P, s, nd, parity_mA(P->m), j, jbar);
    memcpy(jbar + n, j + n, 2 * n * sizeof(cplx));
    return 0;
}

/* Current correction (section 3.7), on the staged current jbar (J_rho on the staggered rho grid, J_theta,
 * J_z) with the planar density differential rho_xy of the same mode:
 *   d = rho_xy - D_div^(+,mS) Jbar_rho - (i m / rho) Jbar_theta        (primary rows)
 *   [L_rho^(mS) - m^2 / rho^2] phi = d                                  (one solve per z column)
 *   Jbar_rho += D_rho^(-,mS) phi (rows k >= 1),  Jbar_theta += (i m / rho) phi,  Jbar_z unchanged.
 * The radial operator is the one of the envelope (centred second and first differences, section 2.3);
 * its matrix is built by applying it to unit vectors, and each column is solved by Gaussian elimination
 * with partial pivoting.  In place on jbar. */
int oracle_correct_current(const oracle_problem *P, double complex *jbar, const double complex *rho_xy)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2, m = P->m, nr = P->nr, nz = P->nz;
    const size_t n = (size_t)nr * nz;
    double a[16], b[17], d1[16];
    oracle_coef_staggered(nd, a);
    oracle_coef_centred_d2(nd, b);
    oracle_coef_centred_d1(nd, d1);
    const int pS = parity_mS(m);
    cplx *dv = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx)), *e = malloc(n * sizeof(cplx));
    double *A = malloc((size_t)nr * nr * sizeof(double));
    cplx *x = malloc((size_t)nr * sizeof(cplx));
    double *M = malloc((size_t)nr * nr * sizeof(double));
    if (!dv || !t || !e || !A || !x || !M) return -2;
    /* planar divergence error */
    op_div_plus(P, a, nd, pS, jbar, dv);
    for (int k = 0; k < nr; ++k)
        for (int i = 0; i < nz; ++i) {
            const size_t q = IDX(P, k, i);
            dv[q] = rho_xy[q] - dv[q] - (I * m / ((k + 0.5) * P->dr)) * jbar[n + q];
        }
    /* matrix of L_rho - m^2/rho^2, column kk = the operator on the unit vector of row kk */
    for (int kk = 0; kk < nr; ++kk) {
        memset(e, 0, n * sizeof(cplx));
        for (int i = 0; i < nz; ++i) e[IDX(P, kk, i)] = 1.0;
        op_lap_rho(P, b, d1, nd, pS, e, t);
        for (int k = 0; k < nr; ++k) {
            const double rho = (k + 0.5) * P->dr;
            A[(size_t)k * nr + kk] = creal(t[IDX(P, k, 0)]) - (k == kk ? (double)m * m / (rho * rho) : 0.0);
        }
    }
    /* phi = A^-1 d per column (Gaussian elimination, partial pivoting), kept in t */
    for (int i = 0; i < nz; ++i) {
        memcpy(M, A, (size_t)nr * nr * sizeof(double));
        for (int k = 0; k < nr; ++k) x[k] = dv[IDX(P, k, i)];
        for (int c = 0; c < nr; ++c) {
            int piv = c;
            for (int r = c + 1; r < nr; ++r)
                if (fabs(M[(size_t)r * nr + c]) > fabs(M[(size_t)piv * nr + c])) piv = r;
            if (piv != c) {
                for (int q = 0; q < nr; ++q) {
                    const double tmp = M[(size_t)c * nr + q];
                    M[(size_t)c * nr + q] = M[(size_t)piv * nr + q];
                    M[(size_t)piv * nr + q] = tmp;
                }
                const cplx tx = x[c];
                x[c] = x[piv];
                x[piv] = tx;
            }
            for (int r = c + 1; r < nr; ++r) {
                const double f = M[(size_t)r * nr + c] / M[(size_t)c * nr + c];
                if (f == 0.0) continue;
                for (int q = c; q < nr; ++q) M[(size_t)r * nr + q] -= f * M[(size_t)c * nr + q];
                x[r] -= f * x[c];
            }
        }
        for (int c = nr - 1; c >= 0; --c) {
            cplx v = x[c];
            for (int q = c + 1; q < nr; ++q) v -= M[(size_t)c * nr + q] * x[q];
            x[c] = v / M[(size_t)c * nr + c];
        }
        for (int k = 0; k < nr; ++k) t[IDX(P, k, i)] = x[k];
    }
    /* corrected currents */
    op_dr_minus(P, a, nd, pS, t, e);
    for (int k = 0; k < nr; ++k)
        for (int i = 0; i < nz; ++i) {
            const size_t q = IDX(P, k, i);
            if (k >= 1) jbar[q] += e[q];
            jbar[n + q] += (I * m / ((k + 0.5) * P->dr)) * t[q];
        }
    free(dv); free(t); free(e); free(A); free(x); free(M);
    return 0;
}

static int step_impl(const oracle_problem *P, double complex *psi, const double complex *j, int64_t j_stride,
                     int n_steps, int corrected);

/* One or more midpoint exponential steps (section 2.1 midpoint solution, Taylor sums of
 * section 2.5):  psi' = sum_n (dt^n/n!) H^n psi  -  dt * sum_n ((dt/2)^n/n!) H^n Jbar. */
int oracle_step(const oracle_problem *P, double complex *psi, const double complex *j,
                int64_t j_stride, int n_steps)
{
    return step_impl(P, psi, j, j_stride, n_steps, 0);
}

/* The same with the current correction of section 3.7 applied to Jbar every step; a block of j holds
 * four planes: J_rho, J_theta, J_z and the planar density differential rho_xy. */
int oracle_step_corrected(const oracle_problem *P, double complex *psi, const double complex *j,
                          int64_t j_stride, int n_steps)
{
    return step_impl(P, psi, j, j_stride, n_steps, 1);
}

static int step_impl(const oracle_problem *P, double complex *psi, const double complex *j, int64_t j_stride,
                     int n_steps, int corrected)
{
    if (check_problem(P) || P->taylor_order < 1 || n_steps < 0) return -1;
    const size_t n = (size_t)P->nr * P->nz, n6 = 6 * n;
    const int N = P->taylor_order;
    const double dt = P->dt;
    cplx *term = malloc(n6 * sizeof(cplx));
    cplx *next = malloc(n6 * sizeof(cplx));
    cplx *sum = malloc(n6 * sizeof(cplx));
    cplx *usum = malloc(n6 * sizeof(cplx));
    for (int step = 0; step < n_steps; ++step) {
        /* source-free series  S = sum_n t_n,  t_0 = psi,  t_n = (dt/n) H t_{n-1} */
        memcpy(term, psi, n6 * sizeof(cplx));
        memcpy(sum, psi, n6 * sizeof(cplx));
        for (int k = 1; k <= N; ++k) {
            oracle_apply_H(P, term, next);
            for (size_t q = 0; q < n6; ++q) {
                term[q] = (dt / k) * next[q];
                sum[q] += term[q];
            }
        }
        if (j) {
            /* source series  U = sum_n u_n,  u_0 = (Jbar, 0),  u_n = (dt/(2n)) H u_{n-1} */
            const cplx *js = j + (size_t)(j_stride * step);
            memset(term, 0, n6 * sizeof(cplx));
            oracle_stage_current(P, js, term);
            if (corrected) oracle_correct_current(P, term, js + 3 * n);
            memcpy(usum, term, n6 * sizeof(cplx));
            for (int k = 1; k <= N; ++k) {
                oracle_apply_H(P, term, next);
                for (size_t q = 0; q < n6; ++q) {
                    term[q] = (dt / (2.0 * k)) * next[q];
                    usum[q] += term[q];
                }
            }
            for (size_t q = 0; q < n6; ++q) sum[q] -= dt * usum[q];
        }
        memcpy(psi, sum, n6 * sizeof(cplx));
        oracle_set_axis(P, psi);
    }
    free(term);
    free(next);
    free(sum);
    free(usum);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Laser envelope (section 4): d/dt a = a~, d/dt a~ = (L_rho + L_z - m^2/rho^2 - chi) a             */
/*                                        + 2 i k0 D_z^(C) a + 2 i k0 a~                          */
/* (the complex envelope equation of section 4.1; a is scalar-like, radial symmetry mS).            */
/* ------------------------------------------------------------------------------------------ */

int oracle_apply_Ha(const oracle_problem *P, const double complex *a, const double complex *at,
                    const double *chi, double complex *out_a, double complex *out_at)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2, m = P->m;
    const size_t n = (size_t)P->nr * P->nz;
    double b[17], d[16];
    oracle_coef_centred_d2(nd, b);
    oracle_coef_centred_d1(nd, d);
    cplx *lr = malloc(n * sizeof(cplx)), *lz = malloc(n * sizeof(cplx)), *dz = malloc(n * sizeof(cplx));
    op_lap_rho(P, b, d, nd, parity_mS(m), a, lr);
    op_lap_z(P, b, nd, a, lz);
    op_dz_centred(P, d, nd, a, dz);
    for (int k = 0; k < P->nr; ++k) {
        double rho = (k + 0.5) * P->dr;
        for (int i = 0; i < P->nz; ++i) {
            size_t q = IDX(P, k, i);
            out_a[q] = at[q];
            out_at[q] = lr[q] + lz[q] - ((double)m * m / (rho * rho)) * a[q] - chi[q] * a[q]
                        + 2.0 * I * P->k0 * dz[q] + 2.0 * I * P->k0 * at[q];
        }
    }
    free(lr);
    free(lz);
    free(dz);
    return 0;
}

/* psi_a' = sum_{n=0..N} (dt^n/n!) H_a^n psi_a with chi held at its mid-step value (section 4.1). */
int oracle_envelope_step(const oracle_problem *P, double complex *a, double complex *at,
                         const double *chi, int n_steps)
{
    if (check_problem(P) || P->taylor_order < 1 || n_steps < 0) return -1;
    const size_t n = (size_t)P->nr * P->nz;
    const int N = P->taylor_order;
    cplx *ta = malloc(n * sizeof(cplx)), *tt = malloc(n * sizeof(cplx));
    cplx *na = malloc(n * sizeof(cplx)), *nt = malloc(n * sizeof(cplx));
    cplx *sa = malloc(n * sizeof(cplx)), *st = malloc(n * sizeof(cplx));
    for (int step = 0; step < n_steps; ++step) {
        memcpy(ta, a, n * sizeof(cplx));
        memcpy(tt, at, n * sizeof(cplx));
        memcpy(sa, a, n * sizeof(cplx));
        memcpy(st, at, n * sizeof(cplx));
        for (int k = 1; k <= N; ++k) {
            oracle_apply_Ha(P, ta, tt, chi, na, nt);
            for (size_t q = 0; q < n; ++q) {
                ta[q] = (P->dt / k) * na[q];
                tt[q] = (P->dt / k) * nt[q];
                sa[q] += ta[q];
                st[q] += tt[q];
            }
        }
        memcpy(a, sa, n * sizeof(cplx));
        memcpy(at, st, n * sizeof(cplx));
    }
    free(ta); free(tt); free(na); free(nt); free(sa); free(st);
    return 0;
}

/* Ponderomotive field of the envelope model (section 4.3): with the intensity envelope |a|^2 on the
 * primary grid (m = 0, scalar-like), A~_rho = -D_rho^(-,mS) |a|^2 on the staggered rho rows k >= 1 (row 0:
 * 0) and A~_z = -D_z^(-) |a|^2 on the staggered z points.  out: 3 real planes |a|^2, A~_rho, A~_z. */
int oracle_ponderomotive(const oracle_problem *P, const double complex *a, double *out)
{
    if (check_problem(P) || P->m != 0) return -1;
    const int nd = P->fd_order / 2;
    const size_t n = (size_t)P->nr * P->nz;
    double c[16];
    oracle_coef_staggered(nd, c);
    cplx *i2 = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    if (!i2 || !t) return -2;
    for (size_t q = 0; q < n; ++q) i2[q] = creal(a[q]) * creal(a[q]) + cimag(a[q]) * cimag(a[q]);
    for (size_t q = 0; q < n; ++q) out[q] = creal(i2[q]);
    op_dr_minus(P, c, nd, parity_mS(P->m), i2, t);
    for (size_t q = 0; q < n; ++q) out[n + q] = -creal(t[q]);
    op_dz_minus(P, c, nd, i2, t);
    for (size_t q = 0; q < n; ++q) out[2 * n + q] = -creal(t[q]);
    free(i2);
    free(t);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Scalar absorbing layer (appendix on the scalar absorbing layer, applied to the envelope state as */
/* section 4.2 allows): the damped wave equation with sigma = sigma_z(z) + sigma_rho(rho) is split   */
/* symmetrically as exp(-sigma dt/4) exp(dt H) exp(-sigma dt/4), where H is the undamped operator     */
/* with sigma^2 merged into the susceptibility (chi~ = chi + sigma^2).                               */
/* ------------------------------------------------------------------------------------------ */

/* Layer functions (reading: the companion paper that defines them is not available): polynomial grading
 * sigma_max * d^power with d = depth into the layer in cells / width, d = 1 on the outermost cell; layers
 * of lz columns at both z ends and lr rows at the outer rho edge, none at the axis.  sigma is [nr][nz]. */
int oracle_absorber_profile(const oracle_problem *P, int lz, int lr, double sigma_max, double power,
                            double *sigma)
{
    if (check_problem(P) || lz < 0 || lr < 0 || 2 * lz > P->nz || lr > P->nr || !(sigma_max >= 0.0)) return -1;
    for (int k = 0; k < P->nr; ++k) {
        double sr = 0.0;
        if (lr > 0 && k >= P->nr - lr) sr = sigma_max * pow((double)(k - (P->nr - 1 - lr)) / lr, power);
        for (int i = 0; i < P->nz; ++i) {
            double sz = 0.0;
            if (lz > 0 && i < lz) sz = sigma_max * pow((double)(lz - i) / lz, power);
            if (lz > 0 && i >= P->nz - lz) sz = sigma_max * pow((double)(i - (P->nz - 1 - lz)) / lz, power);
            sigma[IDX(P, k, i)] = sz + sr;
        }
    }
    return 0;
}

/* n_steps of psi_a' = exp(-sigma dt/4) T_N(dt H_a(chi + sigma^2)) exp(-sigma dt/4) psi_a. */
int oracle_envelope_step_absorbing(const oracle_problem *P, double complex *a, double complex *at,
                                   const double *chi, const double *sigma, int n_steps)
{
    if (check_problem(P) || n_steps < 0) return -1;
    const size_t n = (size_t)P->nr * P->nz;
    double *chit = malloc(n * sizeof(double)), *damp = malloc(n * sizeof(double));
    for (size_t q = 0; q < n; ++q) {
        chit[q] = chi[q] + sigma[q] * sigma[q];
        damp[q] = exp(-sigma[q] * P->dt / 4.0);
    }
    int rc = 0;
    for (int step = 0; step < n_steps && !rc; ++step) {
        for (size_t q = 0; q < n; ++q) {
            a[q] *= damp[q];
            at[q] *= damp[q];
        }
        rc = oracle_envelope_step(P, a, at, chit, 1);
        for (size_t q = 0; q < n; ++q) {
            a[q] *= damp[q];
            at[q] *= damp[q];
        }
    }
    free(chit);
    free(damp);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Diagnostics (section 5.1): energy integral of |E|^2 + |B|^2 over the volume and its z-centroid.  */
/* The theta integral of a complex mode gives 2 pi |F|^2 for m = 0 and pi |F|^2 for m >= 1.          */
/* ------------------------------------------------------------------------------------------ */

void oracle_energy(const oracle_problem *P, const double complex *psi, double *energy, double *zc)
{
    const size_t n = (size_t)P->nr * P->nz;
    const double w = (P->m == 0) ? 2.0 * M_PI : M_PI;
    /* staggering per component (Table 1): rho-staggered and z-staggered flags */
    static const int rst[6] = {1, 0, 0, 0, 1, 1};
    static const int zst[6] = {0, 0, 1, 1, 1, 0};
    double W = 0.0, Wz = 0.0;
    for (int f = 0; f < 6; ++f)
        for (int k = 0; k < P->nr; ++k) {
            double r = rst[f] ? k * P->dr : (k + 0.5) * P->dr;
            for (int i = 0; i < P->nz; ++i) {
                double z = zst[f] ? (i - 0.5) * P->dz : i * P->dz;
                cplx F = psi[f * n + IDX(P, k, i)];
                double e = w * r * P->dr * P->dz * (creal(F) * creal(F) + cimag(F) * cimag(F));
                W += e;
                Wz += z * e;
            }
        }
    *energy = W;
    *zc = (W > 0.0) ? Wz / W : 0.0;
}

void oracle_envelope_energy(const oracle_problem *P, const double complex *a,
                            const double complex *at, double *energy, double *zc)
{
    const double w = (P->m == 0) ? 2.0 * M_PI : M_PI;
    double W = 0.0, Wz = 0.0;
    for (int k = 0; k < P->nr; ++k) {
        double r = (k + 0.5) * P->dr;
        for (int i = 0; i < P->nz; ++i) {
            cplx e = at[IDX(P, k, i)] - I * P->k0 * a[IDX(P, k, i)];
            double v = w * r * P->dr * P->dz * (creal(e) * creal(e) + cimag(e) * cimag(e));
            W += v;
            Wz += i * P->dz * v;
        }
    }
    *energy = W;
    *zc = (W > 0.0) ? Wz / W : 0.0;
}

/* ---------------------------------------------------------------------------------------------------
 * Deposition of point samples (sections 3.2, 3.5, 3.6), the source of the prescribed bunch current.
 * A sample is (z, x, y, q w); it moves with velocity vz along z (no transverse motion).
 * ------------------------------------------------------------------------------------------------- */

/* Cubic B-spline particle shape (3rd order) of a distance x in cells; its integer shifts sum to 1. */
static double bspline3(double x)
{
    x = fabs(x);
    if (x < 1.0) return 2.0 / 3.0 - x * x + 0.5 * x * x * x;
    if (x < 2.0) {
        const double t = 2.0 - x;
        return t * t * t / 6.0;
    }
    return 0.0;
}

/* Sign with which the part of a sample's radial shape at rho < 0 is folded back (section 3.5): the
 * component's m_S or m_A type for m = 0, 1, and antisymmetric for every m > 1, so that a sample on the axis
 * deposits nothing into those modes. */
static int fold_mS(int m) { return m > 1 ? -1 : parity_mS(m); }
static int fold_mA(int m) { return m > 1 ? -1 : parity_mA(m); }

/* Quadrature weights of the radial integral from the axis on the primary rows (section 3.5). */
static double h_weight(int k) { return k == 0 ? 7.0 / 8.0 : (k == 1 ? 73.0 / 72.0 : 1.0); }

/* Radial shape of section 3.5 of a sample at rho_p on primary row k >= 0 (rho_k = (k + 1/2) dr), with
 * the part at rho < 0 folded back onto row k with the sign p of fold_mS / fold_mA (the mirror rule of
 * section 3.5 applied to the shape):
 *   N^-1 rho_k^(eps - 1) (w_k + p w_(-1-k)),   w_j = S3((rho_j - rho_p) / dr),
 *   N = sum_(k >= 0) h_k rho_k^eps (w_k + w_(-1-k)) dr   (the sample's shape on the folded grid). */
static double radial_norm(const oracle_problem *P, double rho_p, double eps)
{
    double N = 0.0;
    for (int k = 0; (k + 0.5) * P->dr < rho_p + 3.0 * P->dr; ++k) {
        const double rk = (k + 0.5) * P->dr;
        const double w = bspline3((rk - rho_p) / P->dr) + bspline3((-rk - rho_p) / P->dr);
        N += h_weight(k) * pow(rk, eps) * w * P->dr;
    }
    return N;
}
static double radial_shape(const oracle_problem *P, double rho_p, double eps, double N, int parity, int k)
{
    const double rk = (k + 0.5) * P->dr;
    const double w = bspline3((rk - rho_p) / P->dr) + parity * bspline3((-rk - rho_p) / P->dr);
    return pow(rk, eps - 1.0) * w / N;
}

/* Angular shape of section 3.2, deposition form (l = 1), as the complex mode coefficient of the
 * convention F = Re sum_m F_m e^(i m theta) (a reading of the normalisation): 1/(2 pi) for m = 0,
 * e^(-i m theta_p)/pi else. */
static cplx angular_shape(int m, double theta)
{
    if (m == 0) return 1.0 / (2.0 * M_PI);
    return (cos(m * theta) - I * sin(m * theta)) / M_PI;
}

/* A sample is deposited only when its z shape lies on grid nodes: nodes floor(z/dz) - 1 .. floor(z/dz) + 2
 * inside [0, nz) (for the current: for both positions z -+ vz dt/2).  Charge entering or leaving at a z
 * end would otherwise show up in the integrated shape as a current along the whole grid. */
static int z_inside(const oracle_problem *P, double zc)
{
    return floor(zc) - 1 >= 0 && floor(zc) + 2 <= P->nz - 1;
}

/* Charge density of mode m (m_S fold) of the samples shifted by dz_shift along z, added into rho. */
int oracle_deposit_rho(const oracle_problem *P, const double *samples, long n, double dz_shift, double eps,
                       double complex *rho)
{
    if (check_problem(P) || !samples || !rho || n < 0) return -1;
    const int nz = P->nz, nr = P->nr, p = fold_mS(P->m);
    for (long s = 0; s < n; ++s) {
        const double z = samples[4 * s] + dz_shift, x = samples[4 * s + 1], y = samples[4 * s + 2];
        if (!z_inside(P, z / P->dz)) continue;
        const double qw = samples[4 * s + 3];
        const double rho_p = sqrt(x * x + y * y);
        const double N = radial_norm(P, rho_p, eps);
        const cplx ang = angular_shape(P->m, atan2(y, x));
        for (int k = 0; k < nr; ++k) {
            const double rs = radial_shape(P, rho_p, eps, N, p, k);
            if (rs == 0.0) continue;
            for (int i = 0; i < nz; ++i) {
                const double sz = bspline3(i - z / P->dz) / P->dz;
                if (sz != 0.0) rho[(size_t)k * nz + i] += qw * sz * rs * ang;
            }
        }
    }
    return 0;
}

/* Longitudinal current of section 3.6 (samples moving with vz, no transverse motion), added into plane
 * 2 of j (3 planes J_rho, J_theta, J_z; J_z on the z-staggered points z_i - dz/2).  The integrated shape
 * F(i) = sum_(i' < i) S3(i' - z/dz) of the positions z -+ vz dt/2 gives, from the discrete continuity
 * equation (a reading of section 3.6),  J_z(i - 1/2) = q w (F_-(i) - F_+(i)) / dt * radial shape * angular shape. */
int oracle_deposit_jz(const oracle_problem *P, const double *samples, long n, double vz, double eps,
                      double complex *j)
{
    if (check_problem(P) || !samples || !j || n < 0 || !(P->dt > 0)) return -1;
    const int nz = P->nz, nr = P->nr, p = fold_mS(P->m);
    double complex *jz = j + 2 * (size_t)nz * nr;
    double *dF = malloc(sizeof(double) * (size_t)nz);
    if (!dF) return -2;
    for (long s = 0; s < n; ++s) {
        const double z = samples[4 * s], x = samples[4 * s + 1], y = samples[4 * s + 2];
        const double qw = samples[4 * s + 3];
        const double zp = (z + 0.5 * vz * P->dt) / P->dz, zm = (z - 0.5 * vz * P->dt) / P->dz;
        if (!z_inside(P, zp) || !z_inside(P, zm)) continue;
        /* F(i) over nodes i' < i; outside nodes lo .. hi both shapes are wholly left or wholly right of
         * i - 1/2, so F_- = F_+ there and the current is zero */
        const int lo = (int)floor(fmin(zp, zm)) - 1, hi = (int)floor(fmax(zp, zm)) + 2;
        double Fp = 0.0, Fm = 0.0;
        for (int i = 0; i < nz; ++i) {
            dF[i] = (i >= lo && i <= hi) ? (Fm - Fp) / P->dt : 0.0;
            Fp += bspline3(i - zp);
            Fm += bspline3(i - zm);
        }
        const double rho_p = sqrt(x * x + y * y);
        const double N = radial_norm(P, rho_p, eps);
        const cplx ang = angular_shape(P->m, atan2(y, x));
        for (int k = 0; k < nr; ++k) {
            const double rs = radial_shape(P, rho_p, eps, N, p, k);
            if (rs == 0.0) continue;
            for (int i = 0; i < nz; ++i)
                if (dF[i] != 0.0) jz[(size_t)k * nz + i] += qw * dF[i] * rs * ang;
        }
    }
    free(dF);
    return 0;
}

/* Currents of moving samples (section 3.6): samples hold z, x, y, q w, v_x, v_y, v_z and one unused word.
 * Positions z+-, x+-, y+- = position +- v dt/2 give rho+-, theta+-.  Added into j (planes J_rho, J_theta,
 * J_z) and, when rho_xy is not NULL, into the planar density differential of section 3.7:
 *   J_rho   += q w v_rho S(z_p) R_A(rho_p) A(theta_p),  J_theta += q w v_theta S(z_p) R_A(rho_p) A(theta_p)
 *   J_z(i - 1/2) += q w (F_-(i) - F_+(i)) / dt * (R_S(rho+) A(theta+) + R_S(rho-) A(theta-)) / 2
 *   rho_xy  += q w (S(z+) + S(z-)) / 2 * (R_S(rho+) A(theta+) - R_S(rho-) A(theta-)) / dt
 * with S(z) = S3(i - z/dz)/dz, F_+- the integrated z shape of z+- (as for oracle_deposit_jz), R_A / R_S the
 * radial shape folded with the m_A (polar components) / m_S (z component, densities) parity, A the angular
 * shape; v_rho = (x v_x + y v_y)/rho, v_theta = (x v_y - y v_x)/rho at the sample (0 on the axis).  A sample
 * whose z shapes at z+- reach past a z end is not deposited.  The integrated shape of section 3.6 spans
 * every node between the two positions, however far apart they are. */
int oracle_deposit_current(const oracle_problem *P, const double *samples, long n, double eps, double complex *j,
                           double complex *rho_xy)
{
    if (check_problem(P) || !samples || !j || n < 0 || !(P->dt > 0)) return -1;
    const int nz = P->nz, nr = P->nr, pS = fold_mS(P->m), pA = fold_mA(P->m);
    const size_t np = (size_t)nz * nr;
    double *dF = malloc(sizeof(double) * (size_t)nz);
    if (!dF) return -2;
    for (long s = 0; s < n; ++s) {
        const double *q = samples + 8 * s;
        const double z = q[0], x = q[1], y = q[2], qw = q[3], vx = q[4], vy = q[5], vz = q[6];
        const double h = 0.5 * P->dt;
        const double zp = (z + h * vz) / P->dz, zm = (z - h * vz) / P->dz;
        if (!z_inside(P, zp) || !z_inside(P, zm)) continue;
        const double xp = x + h * vx, yp = y + h * vy, xm = x - h * vx, ym = y - h * vy;
        const double rp = sqrt(xp * xp + yp * yp), rm = sqrt(xm * xm + ym * ym), r0 = sqrt(x * x + y * y);
        const cplx ap = angular_shape(P->m, atan2(yp, xp)), am = angular_shape(P->m, atan2(ym, xm));
        const cplx a0 = angular_shape(P->m, atan2(y, x));
        const double vr = r0 > 0 ? (x * vx + y * vy) / r0 : 0.0, vt = r0 > 0 ? (x * vy - y * vx) / r0 : 0.0;
        const double Np = radial_norm(P, rp, eps), Nm = radial_norm(P, rm, eps), N0 = radial_norm(P, r0, eps);
        double Fp = 0.0, Fm = 0.0;
        for (int i = 0; i < nz; ++i) {
            dF[i] = (Fm - Fp) / P->dt;
            Fp += bspline3(i - zp);
            Fm += bspline3(i - zm);
        }
        for (int k = 0; k < nr; ++k) {
            const double RA = radial_shape(P, r0, eps, N0, pA, k);
            const cplx tp = radial_shape(P, rp, eps, Np, pS, k) * ap, tm = radial_shape(P, rm, eps, Nm, pS, k) * am;
            for (int i = 0; i < nz; ++i) {
                const size_t o = IDX(P, k, i);
                const double s0 = bspline3(i - z / P->dz) / P->dz;
                if (s0 != 0.0 && RA != 0.0) {
                    j[o] += qw * vr * s0 * RA * a0;
                    j[np + o] += qw * vt * s0 * RA * a0;
                }
                if (dF[i] != 0.0) j[2 * np + o] += qw * dF[i] * 0.5 * (tp + tm);
                if (rho_xy) {
                    const double sz = 0.5 * (bspline3(i - zp) + bspline3(i - zm)) / P->dz;
                    if (sz != 0.0) rho_xy[o] += qw * sz * (tp - tm) / P->dt;
                }
            }
        }
    }
    free(dF);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Field interpolation (section 3.3): destaggering to the primary grids, then the sum of the shapes   */
/* of the sample over the nodes, the radial shape treated as a Cartesian one.                          */
/* ------------------------------------------------------------------------------------------ */

/* The six components on the primary grids: E_rho^(C) = S_rho^(+,mA) E_rho, E_theta as it is,
 * E_z^(C) = S_z^(+) E_z, B_rho^(C) = S_z^(+) B_rho, B_theta^(C) = S_rho^(+,mA) S_z^(+) B_theta,
 * B_z^(C) = S_rho^(+,mS) B_z.  The staggered operands' axis values follow the boundary rule. */
int oracle_destagger(const oracle_problem *P, const double complex *psi, double complex *out)
{
    if (check_problem(P)) return -1;
    const int nd = P->fd_order / 2, m = P->m;
    const size_t n = (size_t)P->nr * P->nz;
    double s[16], c[16];
    oracle_coef_halfshift(nd, s);
    oracle_coef_axis(nd, c);
    const int pS = parity_mS(m), pA = parity_mA(m);
    cplx *t = malloc(n * sizeof(cplx));
    if (!t) return -2;
    op_shift_plus_rho(P, s, c, nd, pA, m == 1, psi + ER * n, out + ER * n);
    memcpy(out + ETH * n, psi + ETH * n, n * sizeof(cplx));
    op_shift_plus_z(P, s, nd, psi + EZ * n, out + EZ * n);
    op_shift_plus_z(P, s, nd, psi + BR * n, out + BR * n);
    op_shift_plus_z(P, s, nd, psi + BTH * n, t);
    op_shift_plus_rho(P, s, c, nd, pA, m == 1, t, out + BTH * n);
    op_shift_plus_rho(P, s, c, nd, pS, m == 0, psi + BZ * n, out + BZ * n);
    free(t);
    return 0;
}

/* Adds to fields[s][c] (n x 6, E_rho, E_theta, E_z, B_rho, B_theta, B_z) the value of mode m at sample s:
 *   Re( e^(i m theta_p) sum_(i,k) S3(i - z_p/dz) S3((rho_k - rho_p)/drho) F_c(k, i) )
 * over the extended primary grid rho_k = (k + 1/2) drho: rows k < 0 take the parity times row -1-k
 * (mA for the rho and theta components, mS for the z components), rows >= nr and columns outside [0, nz)
 * are 0.  `prim` holds the six destaggered planes. */
int oracle_interpolate(const oracle_problem *P, const double complex *prim, const double *samples, long n,
                       double *fields)
{
    if (check_problem(P) || n < 0) return -1;
    const size_t np = (size_t)P->nr * P->nz;
    const int pS = parity_mS(P->m), pA = parity_mA(P->m);
    const int par[6] = {pA, pA, pS, pA, pA, pS};
    for (long s = 0; s < n; ++s) {
        const double z = samples[4 * s], x = samples[4 * s + 1], y = samples[4 * s + 2];
        const double rho = sqrt(x * x + y * y), th = atan2(y, x);
        const cplx rot = cexp(I * (double)P->m * th);
        for (int f = 0; f < 6; ++f) {
            cplx v = 0.0;
            for (int k = -P->nr; k < P->nr; ++k) {
                const double wr = bspline3(((k + 0.5) * P->dr - rho) / P->dr);
                if (wr == 0.0) continue;
                for (int i = 0; i < P->nz; ++i) {
                    const double wz = bspline3(i - z / P->dz);
                    if (wz != 0.0) v += wz * wr * prim_val(P, prim + f * np, par[f], k, i);
                }
            }
            fields[6 * s + f] += creal(v * rot);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* 2x supersampled interpolation (section 3.4: the fields' resolution is doubled before the shape */
/* sum, along z, rho or both).  Reading: the doubled grid of a component is the union of the two  */
/* position sets of the Yee layout along that direction, primary and staggered, the missing set   */
/* filled by the same-order Lagrange half shift (S^(+) towards primary, S^(-) towards staggered), */
/* and the cubic shape is taken in units of the doubled grid's spacing.                           */
/* ------------------------------------------------------------------------------------------ */

/* S_z^(-): primary z -> staggered z, value at (i - 1/2) dz from columns i + j - 1 and i - j. */
static void op_shift_minus_z(const oracle_problem *P, const double *s_, int nd, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += s_[j - 1] * (prim_val(P, in, +1, k, i + j - 1) + prim_val(P, in, +1, k, i - j));
            out[IDX(P, k, i)] = s;
        }
}

/* S_rho^(-) on every staggered row, the axis included: value at k drho from the primary rows k + j - 1
 * and k - j, rows below the axis mirrored with the parity. */
static void op_shift_minus_rho_all(const oracle_problem *P, const double *s_, int nd, int parity, const cplx *in,
                                   cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nr; ++k)
        for (int i = 0; i < P->nz; ++i) {
            cplx s = 0.0;
            for (int j = 1; j <= nd; ++j)
                s += s_[j - 1] * (prim_val(P, in, parity, k + j - 1, i) + prim_val(P, in, parity, k - j, i));
            out[IDX(P, k, i)] = s;
        }
}

/* Value of component plane set v[zs + 2 rs] (zs, rs = 1: staggered position along z, rho) at row k,
 * column i: 0 outside the grid; on the axis row of a staggered-rho set of a component whose own rho
 * position is staggered, the axis rule of section 2.4 (the stored axis slot is not a value). */
static cplx fine_node(const oracle_problem *P, cplx *const v[4], int own_rs, const double *cax, int nd,
                      int extrapolate, int zs, int rs, int k, int i)
{
    if (i < 0 || i >= P->nz || k >= P->nr) return 0.0;
    const cplx *f = v[zs + 2 * rs];
    if (rs == 1 && k == 0 && own_rs == 1) return axis_value(P, cax, nd, f, i, extrapolate);
    return f[IDX(P, k, i)];
}

int oracle_gather_fine(const oracle_problem *P, const double complex *psi, const double *samples, long n, int ss,
                       double *fields)
{
    if (check_problem(P) || n < 0 || ss < 0 || ss > 3) return -1;
    const int nd = P->fd_order / 2, m = P->m, nz = P->nz, nr = P->nr;
    const size_t np = (size_t)nr * nz;
    double s[16], c[16];
    oracle_coef_halfshift(nd, s);
    oracle_coef_axis(nd, c);
    const int pS = parity_mS(m), pA = parity_mA(m);
    /* own positions (Table 1): z staggered for E_z, B_rho, B_theta; rho staggered for E_rho, B_theta, B_z */
    const int own_z[6] = {0, 0, 1, 1, 1, 0}, own_r[6] = {1, 0, 0, 0, 1, 1};
    const int par[6] = {pA, pA, pS, pA, pA, pS};
    const int extrap[6] = {m == 1, 0, 0, 0, m == 1, m == 0};
    cplx *buf = malloc(6 * 4 * np * sizeof(cplx));
    if (!buf) return -2;
    cplx *v[6][4];
    for (int f = 0; f < 6; ++f) {
        for (int t = 0; t < 4; ++t) v[f][t] = buf + (4 * f + t) * np;
        const int zn = own_z[f], rn = own_r[f], zo = 1 - zn, ro = 1 - rn;
        memcpy(v[f][zn + 2 * rn], psi + f * np, np * sizeof(cplx));
        /* along z first, then along rho (the two commute) */
        if (zn) op_shift_plus_z(P, s, nd, v[f][zn + 2 * rn], v[f][zo + 2 * rn]);
        else op_shift_minus_z(P, s, nd, v[f][zn + 2 * rn], v[f][zo + 2 * rn]);
        for (int zs = 0; zs < 2; ++zs) {
            if (rn) op_shift_plus_rho(P, s, c, nd, par[f], extrap[f], v[f][zs + 2 * rn], v[f][zs + 2 * ro]);
            else op_shift_minus_rho_all(P, s, nd, par[f], v[f][zs + 2 * rn], v[f][zs + 2 * ro]);
        }
    }
    const int sz = ss & 1, sr = (ss >> 1) & 1;
    for (long q = 0; q < n; ++q) {
        const double z = samples[4 * q], x = samples[4 * q + 1], y = samples[4 * q + 2];
        const double rho = sqrt(x * x + y * y), th = atan2(y, x);
        const cplx rot = cexp(I * (double)m * th);
        /* nodes: along z, u dz/2 (doubled: odd u staggered at column (u+1)/2, even u primary at u/2) or
         * i dz; along rho, g drho/2 (doubled: even g staggered row g/2, odd g primary row (g-1)/2, g < 0
         * the mirror of -g) or (k + 1/2) drho (k < 0 the mirror of row -1-k) */
        const int nzn = sz ? 2 * nz + 1 : nz, nrn = sr ? 2 * nr : nr;
        for (int f = 0; f < 6; ++f) {
            cplx acc = 0.0;
            for (int a = -nrn; a < nrn; ++a) {
                double wr;
                int rs, k, sign = 1;
                if (sr) {
                    wr = bspline3(a - 2.0 * rho / P->dr);
                    int g = a;
                    if (g < 0) {
                        g = -g;
                        sign = par[f];
                    }
                    rs = (g % 2 == 0);
                    k = rs ? g / 2 : (g - 1) / 2;
                } else {
                    wr = bspline3(a + 0.5 - rho / P->dr);
                    rs = 0;
                    k = a;
                    if (k < 0) {
                        k = -1 - k;
                        sign = par[f];
                    }
                }
                if (wr == 0.0) continue;
                for (int b = -1; b < nzn; ++b) {
                    double wz;
                    int zs, i;
                    if (sz) {
                        wz = bspline3(b - 2.0 * z / P->dz);
                        zs = (b % 2 != 0);
                        i = zs ? (b + 1) / 2 : b / 2;
                    } else {
                        wz = bspline3(b - z / P->dz);
                        zs = 0;
                        i = b;
                    }
                    if (wz == 0.0) continue;
                    acc += wz * wr * (double)sign * fine_node(P, v[f], own_r[f], c, nd, extrap[f], zs, rs, k, i);
                }
            }
            fields[6 * q + f] += creal(acc * rot);
        }
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Ponderomotive fields at sample positions (section 4.3: |a|^2 and A~ are interpolated at the      */
/* particles alongside E and B).  The m = 0 planes of oracle_ponderomotive, |a|^2 (primary), A~_rho */
/* (staggered rows, odd in rho, 0 on the axis) and A~_z (staggered columns), are brought to the     */
/* primary grid with S_rho^(+) and S_z^(+) as in oracle_destagger, then interpolated with the cubic */
/* shapes of oracle_interpolate over the grid extended below the axis (|a|^2, A~_z even, A~_rho     */
/* odd); no angular factor (m = 0).  Writes out[3 s + c].                                          */
/* ------------------------------------------------------------------------------------------ */
int oracle_envelope_gather(const oracle_problem *P, const double *pond, const double *samples, long n, double *out)
{
    if (check_problem(P) || P->m != 0 || n < 0) return -1;
    const int nd = P->fd_order / 2;
    const size_t np = (size_t)P->nr * P->nz;
    double s[16], c[16];
    oracle_coef_halfshift(nd, s);
    oracle_coef_axis(nd, c);
    cplx *in = malloc(3 * np * sizeof(cplx)), *prim = malloc(3 * np * sizeof(cplx));
    if (!in || !prim) {
        free(in);
        free(prim);
        return -2;
    }
    for (size_t q = 0; q < 3 * np; ++q) in[q] = pond[q];
    memcpy(prim, in, np * sizeof(cplx));
    op_shift_plus_rho(P, s, c, nd, -1, 0, in + np, prim + np);
    op_shift_plus_z(P, s, nd, in + 2 * np, prim + 2 * np);
    const int par[3] = {+1, -1, +1};
    for (long q = 0; q < n; ++q) {
        const double z = samples[4 * q], x = samples[4 * q + 1], y = samples[4 * q + 2];
        const double rho = sqrt(x * x + y * y);
        for (int f = 0; f < 3; ++f) {
            double v = 0.0;
            for (int k = -P->nr; k < P->nr; ++k) {
                const double wr = bspline3(((k + 0.5) * P->dr - rho) / P->dr);
                if (wr == 0.0) continue;
                for (int i = 0; i < P->nz; ++i) {
                    const double wz = bspline3(i - z / P->dz);
                    if (wz != 0.0) v += wz * wr * creal(prim_val(P, prim + f * np, par[f], k, i));
                }
            }
            out[3 * q + f] = v;
        }
    }
    free(in);
    free(prim);
    return 0;
}
