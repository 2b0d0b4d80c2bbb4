"""Pins of the oracle's banded operators, including the near-axis rows (sections 2.2-2.4).

A staggered difference / half-shift of order 2N_D is exact on polynomials of degree <= 2N_D-1 and the
centred second difference on degree <= 2N_D+1.  With the symmetric / antisymmetric extension of section
2.4, a monomial rho^p extended with sign (-1)^p is the same polynomial on rho < 0, so every row -- the
ones next to the axis included -- must reproduce the analytic derivative.  Rows that would reach past the
outer radial edge (where values are ignored) and past the z ends are excluded.  A mistake in a ghost
index, a parity, an axis value or a grid offset makes the near-axis rows fail.
"""
import numpy as np
import pytest

import oracle
from oracle import (OP_AXIS, OP_DIV_MINUS, OP_DIV_PLUS, OP_DR_MINUS, OP_DR_PLUS, OP_DZ_CENTRED,
                    OP_DZ_MINUS, OP_DZ_PLUS, OP_LAP_RHO, OP_LAP_Z, OP_SHIFT_MINUS)

ORDERS = [2, 4, 6, 8, 12, 16, 24, 32]


def grid(nd, nr=None, nz=6):
    nr = nr or 3 * nd + 4
    # rho spans ~[0, 1.1]: keeps rho^p of modest size for p up to 31
    return oracle.Grid(nz=nz, nr=nr, m=0, fd_order=2 * nd, taylor_order=1, dz=0.1, dr=1.0 / (nr - nd),
                       dt=0.0)


def rho_prim(g):
    return (np.arange(g.nr) + 0.5) * g.dr


def rho_stag(g):
    return np.arange(g.nr) * g.dr


def as_plane(g, col):
    return np.repeat(col[:, None], g.nz, axis=1).astype(np.complex128)


def check_rows(got, want, rows, rtol):
    got = got[rows, 0].real
    want = want[rows]
    scale = max(1.0, np.max(np.abs(want)))
    err = np.max(np.abs(got - want)) / scale
    assert err < rtol, err


def tol(nd, p):
    return 1e-12 * 4.0 ** (max(p, 1) / 4.0) * nd


@pytest.mark.parametrize("order", ORDERS)
def test_dr_minus_exact_on_parity_monomials(order):
    nd = order // 2
    g = grid(nd)
    rows = np.arange(1, g.nr - nd + 1)          # staggered rows k>=1 whose stencil stays inside
    for p in range(0, 2 * nd):
        f = as_plane(g, rho_prim(g) ** p)
        out = oracle.apply_op(g, OP_DR_MINUS, f, parity=(-1) ** p)
        want = p * rho_stag(g) ** (p - 1) if p > 0 else 0 * rho_stag(g)
        check_rows(out, want, rows, tol(nd, p))


@pytest.mark.parametrize("order", ORDERS)
def test_dr_plus_exact_on_parity_monomials(order):
    nd = order // 2
    g = grid(nd)
    rows = np.arange(0, g.nr - nd)              # primary rows, axis-adjacent ones included
    for p in range(0, 2 * nd):
        f = as_plane(g, rho_stag(g) ** p)
        f[0] = 1234.5 + 77j                       # the stored axis slot must never be read
        # constant on the axis (p == 0) needs the extrapolated axis value; odd p are zero there by
        # antisymmetry; even p >= 2 are zero on the axis (the rule used for modes m >= 2).
        for extrap in ([True] if p == 0 else [False, True] if p % 2 == 0 and p <= 2 * nd - 2 else [False]):
            out = oracle.apply_op(g, OP_DR_PLUS, f, parity=(-1) ** p, axis_extrapolate=extrap)
            want = p * rho_prim(g) ** (p - 1) if p > 0 else 0 * rho_prim(g)
            check_rows(out, want, rows, tol(nd, p))


@pytest.mark.parametrize("order", ORDERS)
def test_div_minus_exact(order):
    # D_div^(-) F = rho^-1 d/drho (rho F); F = rho^p, operand rho^(p+1) has parity (-1)^(p+1)
    nd = order // 2
    g = grid(nd)
    rows = np.arange(1, g.nr - nd + 1)
    for p in range(0, 2 * nd - 1):
        f = as_plane(g, rho_prim(g) ** p)
        out = oracle.apply_op(g, OP_DIV_MINUS, f, parity=(-1) ** (p + 1))
        want = (p + 1) * rho_stag(g)[rows] ** (p - 1)
        full = np.zeros(g.nr)
        full[rows] = want
        check_rows(out, full, rows, tol(nd, p))


@pytest.mark.parametrize("order", ORDERS)
def test_div_plus_exact(order):
    nd = order // 2
    g = grid(nd)
    rows = np.arange(0, g.nr - nd)
    for p in range(0, 2 * nd - 1):
        f = as_plane(g, rho_stag(g) ** p)
        f[0] = -99.0 + 5j                          # axis slot: multiplied by rho = 0, never read
        out = oracle.apply_op(g, OP_DIV_PLUS, f, parity=(-1) ** (p + 1))
        want = (p + 1) * rho_prim(g) ** (p - 1)
        check_rows(out, want, rows, tol(nd, p) * 10)


@pytest.mark.parametrize("order", ORDERS)
def test_halfshift_exact(order):
    nd = order // 2
    g = grid(nd)
    rows = np.arange(1, g.nr - nd + 1)
    for p in range(0, 2 * nd):
        f = as_plane(g, rho_prim(g) ** p)
        out = oracle.apply_op(g, OP_SHIFT_MINUS, f, parity=(-1) ** p)
        check_rows(out, rho_stag(g) ** p, rows, tol(nd, p))


@pytest.mark.parametrize("order", ORDERS)
def test_radial_laplacian_exact(order):
    # L_rho rho^p = p^2 rho^(p-2)   (D^2 exact to degree 2N_D+1, D^(C) to 2N_D)
    nd = order // 2
    g = grid(nd)
    rows = np.arange(0, g.nr - nd)
    for p in range(0, 2 * nd + 1):
        f = as_plane(g, rho_prim(g) ** p)
        out = oracle.apply_op(g, OP_LAP_RHO, f, parity=(-1) ** p)
        want = p * p * rho_prim(g) ** (p - 2) if p >= 1 else 0 * rho_prim(g)
        check_rows(out, want, rows, tol(nd, p) * 10)


@pytest.mark.parametrize("order", ORDERS)
def test_axis_extrapolation_exact_on_even_polynomials(order):
    nd = order // 2
    g = grid(nd)
    for q in range(0, nd):
        f = as_plane(g, rho_stag(g) ** (2 * q))
        out = oracle.apply_op(g, OP_AXIS, f, parity=1, axis_extrapolate=True)
        want = 1.0 if q == 0 else 0.0
        assert abs(out[0, 0] - want) < 1e-13 * 10 ** (q / 3), (q, out[0, 0])
        assert np.all(out[1:] == 0)


@pytest.mark.parametrize("order", ORDERS)
def test_z_operators_exact_on_polynomials(order):
    nd = order // 2
    nz = 4 * nd + 8
    g = oracle.Grid(nz=nz, nr=nd + 1, m=0, fd_order=order, taylor_order=1, dz=1.0 / nz, dr=1.0, dt=0.0)
    zp = np.arange(nz) * g.dz
    zs = (np.arange(nz) - 0.5) * g.dz
    inner = np.arange(nd, nz - nd)
    for p in range(0, 2 * nd):
        f = np.repeat((zp ** p)[None, :], g.nr, axis=0).astype(complex)
        out = oracle.apply_op(g, OP_DZ_MINUS, f)
        want = p * zs ** (p - 1) if p else 0 * zs
        assert np.max(np.abs(out[:, inner] - want[inner])) < tol(nd, p) * max(1, np.abs(want).max())
        f = np.repeat((zs ** p)[None, :], g.nr, axis=0).astype(complex)
        out = oracle.apply_op(g, OP_DZ_PLUS, f)
        want = p * zp ** (p - 1) if p else 0 * zp
        inner2 = np.arange(nd - 1, nz - nd)
        assert np.max(np.abs(out[:, inner2] - want[inner2])) < tol(nd, p) * max(1, np.abs(want).max())
    for p in range(0, 2 * nd + 1):
        f = np.repeat((zp ** p)[None, :], g.nr, axis=0).astype(complex)
        out = oracle.apply_op(g, OP_DZ_CENTRED, f)
        want = p * zp ** (p - 1) if p else 0 * zp
        assert np.max(np.abs(out[:, inner] - want[inner])) < tol(nd, p) * 10 * max(1, np.abs(want).max())
        out = oracle.apply_op(g, OP_LAP_Z, f)
        want = p * (p - 1) * zp ** (p - 2) if p >= 2 else 0 * zp
        assert np.max(np.abs(out[:, inner] - want[inner])) < tol(nd, p) * 10 * max(1, np.abs(want).max())


def test_out_of_range_terms_are_ignored():
    # A single nonzero value at the last radial row / last z column: the operators must see zeros
    # beyond the grid (section 2.2), so the row/column just outside contributes nothing.
    nd = 2
    g = oracle.Grid(nz=8, nr=6, m=0, fd_order=4, taylor_order=1, dz=1.0, dr=1.0, dt=0.0)
    f = np.zeros((6, 8), complex)
    f[5, 7] = 1.0
    a = oracle.coef("staggered", nd)
    out = oracle.apply_op(g, OP_DZ_MINUS, f)
    # D_z^(-) at staggered column i uses f_{i+j-1} - f_{i-j}; f_7 enters columns 7 (+a_1) and 6 (+a_2)
    assert np.allclose(out[5], [0, 0, 0, 0, 0, 0, a[1], a[0]])
    out = oracle.apply_op(g, OP_DR_MINUS, f, parity=1)
    assert np.allclose(out[:, 7], [0, 0, 0, 0, a[1], a[0]])


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [4, 8, 16])
def test_current_staging_exact_with_mode_parity(m, order):
    """J_rho of mode m behaves as rho^|m-1| times an even polynomial near the axis (the m_A parity of
    section 2.4), so its half-shift to the rho-staggered rows (the current staging of section 2.5) with m_A mirror ghosts is exact
    on such polynomials up to degree 2N_D - 1, next to the axis included; a current of the other parity
    is not reproduced there.  J_theta and J_z pass through unchanged."""
    nd = order // 2
    g = grid(nd)
    g.m = m
    rows = np.arange(1, g.nr - nd + 1)
    rng = np.random.default_rng(m * 100 + order)
    par = abs(m - 1) % 2
    powers = [p for p in range(0, 2 * nd) if p % 2 == par]
    coef = rng.uniform(-1, 1, len(powers))
    J = np.zeros((3, g.nr, g.nz), np.complex128)
    J[0] = as_plane(g, sum(c * rho_prim(g) ** p for c, p in zip(coef, powers)))
    J[1] = rng.uniform(-1, 1, (g.nr, g.nz)) + 1j * rng.uniform(-1, 1, (g.nr, g.nz))
    J[2] = rng.uniform(-1, 1, (g.nr, g.nz))
    out = oracle.stage_current(g, J)
    check_rows(out[0], sum(c * rho_stag(g) ** p for c, p in zip(coef, powers)), rows, tol(nd, 2 * nd))
    assert np.array_equal(out[1], J[1]) and np.array_equal(out[2], J[2])
    # the other parity: the mirrored ghosts no longer continue the polynomial, row 1 is off
    wrong = np.zeros_like(J)
    wrong[0] = as_plane(g, rho_prim(g) ** (1 - par))
    got = oracle.stage_current(g, wrong)[0][1, 0].real
    assert abs(got - rho_stag(g)[1] ** (1 - par)) > 1e-6
