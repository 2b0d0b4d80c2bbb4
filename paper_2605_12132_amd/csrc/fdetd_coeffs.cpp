// Host-side generation of the finite-difference, interpolation and axis-extrapolation weights used by the
// kernels (sections 2.3 and 2.4 of arXiv 2605.12132: staggered first differences D^(+-), Lagrange half-cell
// shift S^(+-), centred first and second differences D^(C), D^2, and the on-axis extrapolation weights c_k').
//
// All of them are weights of polynomial interpolation at a point, computed here with Fornberg's recursion
// (B. Fornberg, "Generation of finite difference formulas on arbitrarily spaced grids", Math. Comp. 51,
// 1988) in extended precision and rounded once to double.
#include "fdetd_internal.h"

#include <cmath>
#include <vector>

namespace fdetd {

// Weights w[k][j] of the k-th derivative (k <= kmax) at x0 from the values at nodes x[0..n-1].
static void fornberg(const std::vector<long double> &x, long double x0, int kmax,
                     std::vector<std::vector<long double>> &w)
{
    const int n = (int)x.size();
    w.assign(kmax + 1, std::vector<long double>(n, 0.0L));
    w[0][0] = 1.0L;
    long double c1 = 1.0L, c4 = x[0] - x0;
    for (int i = 1; i < n; ++i) {
        const int mn = i < kmax ? i : kmax;
        long double c2 = 1.0L;
        const long double c5 = c4;
        c4 = x[i] - x0;
        for (int j = 0; j < i; ++j) {
            const long double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k)
                    w[k][i] = c1 * (k * w[k - 1][i - 1] - c5 * w[k][i - 1]) / c2;
                w[0][i] = -c1 * c5 * w[0][i - 1] / c2;
            }
            for (int k = mn; k >= 1; --k) w[k][j] = (c4 * w[k][j] - k * w[k - 1][j]) / c3;
            w[0][j] = c4 * w[0][j] / c3;
        }
        c1 = c2;
    }
}

bool make_coefficients(int which, int nd, double *out)
{
    if (nd < 1 || nd > kMaxND) return false;
    std::vector<std::vector<long double>> w;
    std::vector<long double> x;
    switch (which) {
    case COEF_STAGGERED:
    case COEF_HALFSHIFT: {
        // nodes at the half-integer offsets -(nd-1/2) .. (nd-1/2); node index nd-1+j is +(j-1/2)
        for (int j = -nd + 1; j <= nd; ++j) x.push_back(j - 0.5L);
        const int deriv = which == COEF_STAGGERED ? 1 : 0;
        fornberg(x, 0.0L, deriv, w);
        for (int j = 1; j <= nd; ++j) out[j - 1] = (double)w[deriv][nd - 1 + j];
        return true;
    }
    case COEF_CENTRED_D1:
    case COEF_CENTRED_D2: {
        for (int j = -nd; j <= nd; ++j) x.push_back((long double)j);
        const int deriv = which == COEF_CENTRED_D1 ? 1 : 2;
        fornberg(x, 0.0L, deriv, w);
        if (deriv == 1) {
            for (int j = 1; j <= nd; ++j) out[j - 1] = (double)w[1][nd + j];
        } else {
            for (int j = 0; j <= nd; ++j) out[j] = (double)w[2][nd + j];
        }
        return true;
    }
    case COEF_AXIS: {
        // an even function is a polynomial in u = rho^2: extrapolate from u = k^2 (k = 1..nd) to u = 0
        for (int k = 1; k <= nd; ++k) x.push_back((long double)k * k);
        fornberg(x, 0.0L, 0, w);
        for (int k = 1; k <= nd; ++k) out[k - 1] = (double)w[0][k - 1];
        return true;
    }
    default:
        return false;
    }
}

// Largest x such that |T_N(i y)|^2 <= 1 + 2e-9 for every 0 <= y <= x, T_N the degree-N Taylor polynomial of
// exp: the region where the explicit Taylor propagator does not amplify an oscillatory mode.
double taylor_stability_bound(int N)
{
    if (N < 1) return 0.0;
    const long double tol = 2e-9L;
    const long double h = 1e-4L;
    long double y = 0.0L;
    for (; y < 20.0L; y += h) {
        long double re = 0.0L, im = 0.0L, t = 1.0L;  // sum (i y)^n / n!
        for (int n = 0; n <= N; ++n) {
            switch (n & 3) {
            case 0: re += t; break;
            case 1: im += t; break;
            case 2: re -= t; break;
            default: im -= t; break;
            }
            t *= y / (n + 1);
        }
        if (re * re + im * im > 1.0L + tol) break;
    }
    return (double)(y > h ? y - h : 0.0L);
}

}  // namespace fdetd
