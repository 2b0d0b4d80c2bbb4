"""Pins of the oracle's current correction (section 3.7): on the staged current (J_rho staggered), the
planar divergence error d = rho_xy - D_div J_rho - (i m/rho) J_theta is removed by the gradient of phi,
[L_rho - m^2/rho^2] phi = d, J_rho += D_rho^(-) phi, J_theta += (i m/rho) phi.

* a current that already satisfies the planar continuity equation is left unchanged, and J_z always is;
* phi recovered from the theta correction solves the radial equation (the solve and the sign of the
  theta term);
* because L_rho (centred differences) and D_div D_rho^(-) are different discretisations of the same
  operator, the divergence error left after the correction is their consistency error: zero at order 2,
  where the two coincide, and for smooth data falling at the order of the stencils under grid refinement,
  next to the axis included (a wrong sign or parity leaves an O(1) error);
* with a consistent density the corrected step equals the plain step.
"""
import math

import numpy as np
import pytest

import oracle


def grid(m, order, nz, nr, dz, dr):
    return oracle.Grid(nz=nz, nr=nr, m=m, fd_order=order, taylor_order=4, dz=dz, dr=dr, dt=0.5 * dz)


def planar_div(g, jbar):
    """D_div^(+,mS) J_rho + (i m / rho) J_theta on the primary rows (the oracle's own operators)."""
    pS = 1 if g.m % 2 == 0 else -1
    rho = (np.arange(g.nr) + 0.5) * g.dr
    return oracle.apply_op(g, oracle.OP_DIV_PLUS, jbar[0], pS) + (1j * g.m / rho)[:, None] * jbar[1]


def random_staged(g, rng):
    j = rng.standard_normal((3, g.nr, g.nz)) + 1j * rng.standard_normal((3, g.nr, g.nz))
    return oracle.stage_current(g, j)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_consistent_current_is_unchanged(m):
    g = grid(m, 8, 40, 24, 0.3, 0.4)
    rng = np.random.default_rng(m)
    jb = random_staged(g, rng)
    out = oracle.correct_current(g, jb, planar_div(g, jb))
    assert np.max(np.abs(out - jb)) < 1e-12 * np.max(np.abs(jb))
    rng2 = np.random.default_rng(100 + m)
    out2 = oracle.correct_current(g, jb, rng2.standard_normal((g.nr, g.nz)) + 0j)
    assert np.array_equal(out2[2], jb[2])


@pytest.mark.parametrize("m", [1, 2, 3])
def test_phi_solves_the_radial_equation(m):
    g = grid(m, 8, 30, 32, 0.3, 0.4)
    rng = np.random.default_rng(10 + m)
    jb = random_staged(g, rng)
    rxy = rng.standard_normal((g.nr, g.nz)) + 1j * rng.standard_normal((g.nr, g.nz))
    out = oracle.correct_current(g, jb, rxy)
    rho = (np.arange(g.nr) + 0.5) * g.dr
    phi = (out[1] - jb[1]) * (rho / (1j * m))[:, None]
    pS = 1 if m % 2 == 0 else -1
    lhs = oracle.apply_op(g, oracle.OP_LAP_RHO, phi, pS) - (m * m / rho ** 2)[:, None] * phi
    d = rxy - planar_div(g, jb)
    assert np.max(np.abs(lhs - d)) < 1e-9 * np.max(np.abs(d))


def residual_after_correction(m, order, scale):
    """Smooth density of mode m (rho^m near the axis), zero current, grid refined by `scale`; the planar
    divergence error left on the rows away from the outer edge, relative to the density."""
    nd = order // 2
    nz, nr = 8, int(24 * scale) + 4 * nd
    g = grid(m, order, nz, nr, 0.3, 0.25 / scale)
    rho = (np.arange(nr) + 0.5) * g.dr
    rxy = np.repeat((rho ** m * np.exp(-(rho / 2.0) ** 2))[:, None], nz, 1).astype(complex)
    out = oracle.correct_current(g, np.zeros((3, nr, nz), complex), rxy)
    r = rxy - planar_div(g, out)
    rows = rho < 6.0 - 1e-9
    return np.max(np.abs(r[rows])) / np.max(np.abs(rxy))


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_second_order_correction_is_exact(m):
    """At order 2 the centred radial operator is the product D_div^(+) D_rho^(-) row for row (the usual
    three-point cylindrical Laplacian), so the correction removes the divergence error exactly."""
    assert residual_after_correction(m, 2, 1) < 1e-12


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [4, 8])
def test_remaining_divergence_error_converges(m, order):
    e1, e2 = residual_after_correction(m, order, 1), residual_after_correction(m, order, 2)
    rate = math.log2(e1 / e2)
    print(f"m={m} order={order}: residual {e1:.2e} -> {e2:.2e}, rate {rate:.2f}")
    # measured: rate ~ order for even m, ~ order - 1 for odd m (next to the axis)
    assert e1 < 1e-3 and rate > order - 1.5, (e1, e2)


def test_corrected_step_with_consistent_density_equals_plain_step():
    g = grid(1, 8, 60, 24, 0.3, 0.6)
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((6, g.nr, g.nz)) + 1j * rng.standard_normal((6, g.nr, g.nz))
    j = rng.standard_normal((2, 3, g.nr, g.nz)) + 1j * rng.standard_normal((2, 3, g.nr, g.nz))
    j4 = np.zeros((2, 4, g.nr, g.nz), complex)
    for s in range(2):
        j4[s, :3] = j[s]
        j4[s, 3] = planar_div(g, oracle.stage_current(g, j[s]))
    plain = oracle.step(g, psi, j, 2)
    corr = oracle.step_corrected(g, psi, j4, 2)
    assert np.max(np.abs(corr - plain)) < 1e-11 * np.max(np.abs(plain))
