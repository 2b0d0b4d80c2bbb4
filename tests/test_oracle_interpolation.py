"""Pins of the oracle's field interpolation (section 3.3): destaggering with the Lagrange half-shifts
S^(+) and the cubic-shape interpolation at sample positions.

* S_z^(+) is exact on polynomials of degree <= 2 N_D - 1 (away from the z ends);
* S_rho^(+) with the component's parity and axis rule is exact, on every row next to the axis too, on the
  functions the boundary rules describe: rho^q times an even polynomial, q = |m - 1| for the rho and theta
  components (m_A) and q = m for the z components (m_S), degree <= 2 N_D - 2;
* the tensor cubic B-spline reproduces constants and linear functions, and on the extended grid (rows
  below the axis mirrored with the parity) it reproduces odd-parity fields rho (a + b z) next to the axis;
* the angular factor: a mode of constant coefficient F gives Re(F e^(i m theta)) at every angle;
* end to end: a state sampled from such functions on its staggered positions (Table 1) is gathered to the
  exact values at random samples, for m = 0 and m = 1.

2x supersampling (section 3.4), the fields' resolution doubled along z, rho or both before the shape sum:
* the plain case (no direction doubled) is the gather above;
* the same linear fields are gathered exactly, on every component (every chain of half shifts, the
  axis rules and the mirror below the axis of the doubled grid);
* the cubic shape smooths: for a smooth field its sum is f + (h^2/6) f'' + O(h^4) on nodes of spacing h
  (the cubic B-spline's second moment is 1/3), so doubling the resolution must cut the error to a
  quarter of the plain one -- checked against that closed form along z, along rho (through the axis)
  and both.
"""
import math

import numpy as np
import pytest

import oracle

# staggering of the six components (Table 1): rho-staggered, z-staggered
RST = [1, 0, 0, 0, 1, 1]
ZST = [0, 0, 1, 1, 1, 0]
POLAR = [1, 1, 0, 1, 1, 0]  # rho and theta components: m_A; z components: m_S


def grid(m, order, nz=60, nr=30):
    return oracle.Grid(nz=nz, nr=nr, m=m, fd_order=order, taylor_order=4, dz=0.3, dr=0.4, dt=0.1)


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_shift_plus_z_exact_on_polynomials(order):
    nd = order // 2
    g = grid(0, order)
    z_st = (np.arange(g.nz) - 0.5) * g.dz
    z_pr = np.arange(g.nz) * g.dz
    rng = np.random.default_rng(order)
    c = rng.standard_normal(order) * (0.5 ** np.arange(order))
    f = lambda z: sum(ci * (z / 5) ** q for q, ci in enumerate(c))
    plane = np.repeat(f(z_st)[None, :], g.nr, 0).astype(complex)
    out = oracle.apply_op(g, oracle.OP_SHIFT_PLUS_Z, plane)
    cols = slice(nd, g.nz - nd)
    assert np.max(np.abs(out[:, cols] - f(z_pr)[None, cols])) < 1e-12 * np.max(np.abs(f(z_pr)))


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [4, 8, 16])
@pytest.mark.parametrize("polar", [True, False])
def test_shift_plus_rho_exact_near_axis(m, order, polar):
    nd = order // 2
    g = grid(m, order)
    q = abs(m - 1) if polar else m
    parity = (1 if (q % 2 == 0) else -1)
    extrapolate = (m == 1) if polar else (m == 0)
    rng = np.random.default_rng(10 * m + order)
    deg = 2 * nd - 2 - q
    if deg < 0:
        pytest.skip("no polynomial of this parity within the order")
    c = rng.standard_normal(deg // 2 + 1)
    f = lambda r: r ** q * sum(ci * (r / 4) ** (2 * j) for j, ci in enumerate(c))
    r_st = np.arange(g.nr) * g.dr
    r_pr = (np.arange(g.nr) + 0.5) * g.dr
    plane = np.repeat(f(r_st)[:, None], g.nz, 1).astype(complex)
    plane[0] = 123.0  # the axis slot is derived, never read
    out = oracle.apply_op(g, oracle.OP_SHIFT_PLUS_RHO, plane, parity, extrapolate)
    rows = slice(0, g.nr - nd)
    err = np.max(np.abs(out[rows] - f(r_pr)[rows, None]))
    assert err < 1e-12 * max(1.0, np.max(np.abs(f(r_pr)))), err


def samples(rng, n, g, margin_z, max_rho):
    z = rng.uniform(margin_z * g.dz, (g.nz - 1 - margin_z) * g.dz, n)
    r = np.sqrt(rng.uniform(0, max_rho ** 2, n))
    r[: n // 8] = rng.uniform(0, 1.5 * g.dr, n // 8)  # next to the axis
    th = rng.uniform(-math.pi, math.pi, n)
    return np.stack([z, r * np.cos(th), r * np.sin(th), np.ones(n)], axis=1)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_interpolation_reproduces_linear_fields_and_angles(m):
    g = grid(m, 8)
    rng = np.random.default_rng(50 + m)
    s = samples(rng, 400, g, 3, (g.nr - 3) * g.dr)
    z_pr = np.arange(g.nz) * g.dz
    r_pr = (np.arange(g.nr) + 0.5) * g.dr
    F = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))  # F_c = a + b z (even) or rho (a + b z) (odd)
    pS = 1 if m % 2 == 0 else -1
    pA = 1 if abs(m - 1) % 2 == 0 else -1
    odd = [(pA if POLAR[c] else pS) == -1 for c in range(6)]
    prim = np.zeros((6, g.nr, g.nz), complex)
    for c in range(6):
        lin = F[c, 0] + F[c, 1] * z_pr[None, :] / 5
        prim[c] = (r_pr[:, None] if odd[c] else 1.0) * lin
    got = oracle.interpolate(g, prim, s)
    zp, rp = s[:, 0], np.hypot(s[:, 1], s[:, 2])
    th = np.arctan2(s[:, 2], s[:, 1])
    for c in range(6):
        val = (rp if odd[c] else 1.0) * (F[c, 0] + F[c, 1] * zp / 5)
        want = np.real(val * np.exp(1j * m * th))
        assert np.max(np.abs(got[:, c] - want)) < 1e-12, (m, c)


def staggered_state(g, F):
    """State whose component c is a_c + b_c z (even parity) or rho (a_c + b_c z) (odd parity), sampled on
    the component's own staggered positions."""
    pS = 1 if g.m % 2 == 0 else -1
    pA = 1 if abs(g.m - 1) % 2 == 0 else -1
    psi = np.zeros((6, g.nr, g.nz), complex)
    for c in range(6):
        z = (np.arange(g.nz) - 0.5 * ZST[c]) * g.dz
        r = (np.arange(g.nr) + 0.5 * (1 - RST[c])) * g.dr
        odd = (pA if POLAR[c] else pS) == -1
        psi[c] = (r[:, None] if odd else 1.0) * (F[c, 0] + F[c, 1] * z[None, :] / 5)
    return psi


@pytest.mark.parametrize("order", [4, 8, 16])
def test_gather_end_to_end_exact(order):
    """Modes 0 and 1 of one grid, each component a linear field of its parity: destaggering is exact (the
    axis values extrapolate the even components), and the cubic interpolation reproduces the fields."""
    nd = order // 2
    g0, g1 = grid(0, order, nz=80, nr=36), grid(1, order, nz=80, nr=36)
    rng = np.random.default_rng(order)
    F0 = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))
    F1 = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))
    s = samples(rng, 300, g0, nd + 3, (g0.nr - nd - 3) * g0.dr)
    got = oracle.gather([g0, g1], [staggered_state(g0, F0), staggered_state(g1, F1)], s)
    zp, rp = s[:, 0], np.hypot(s[:, 1], s[:, 2])
    th = np.arctan2(s[:, 2], s[:, 1])
    for c in range(6):
        want = 0.0
        for m, F in ((0, F0), (1, F1)):
            pS = 1 if m % 2 == 0 else -1
            pA = 1 if abs(m - 1) % 2 == 0 else -1
            odd = (pA if POLAR[c] else pS) == -1
            want = want + np.real((rp if odd else 1.0) * (F[c, 0] + F[c, 1] * zp / 5) * np.exp(1j * m * th))
        assert np.max(np.abs(got[:, c] - want)) < 1e-11 * max(1.0, np.max(np.abs(want))), (order, c)


def test_supersample_off_is_the_plain_gather():
    g0, g1 = grid(0, 8, nz=50, nr=20), grid(1, 8, nz=50, nr=20)
    rng = np.random.default_rng(7)
    states = [rng.standard_normal((6, 20, 50)) + 1j * rng.standard_normal((6, 20, 50)) for _ in range(2)]
    s = samples(rng, 200, g0, 0, 21 * g0.dr)
    a = oracle.gather([g0, g1], states, s)
    b = oracle.gather_fine([g0, g1], states, s, 0)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("ss", [1, 2, 3])
@pytest.mark.parametrize("order", [4, 8, 16])
def test_supersampled_gather_exact_on_linear_fields(order, ss):
    nd = order // 2
    g0, g1 = grid(0, order, nz=80, nr=36), grid(1, order, nz=80, nr=36)
    rng = np.random.default_rng(100 * ss + order)
    F0 = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))
    F1 = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))
    s = samples(rng, 300, g0, nd + 3, (g0.nr - nd - 3) * g0.dr)
    got = oracle.gather_fine([g0, g1], [staggered_state(g0, F0), staggered_state(g1, F1)], s, ss)
    zp, rp = s[:, 0], np.hypot(s[:, 1], s[:, 2])
    th = np.arctan2(s[:, 2], s[:, 1])
    for c in range(6):
        want = 0.0
        for m, F in ((0, F0), (1, F1)):
            pS = 1 if m % 2 == 0 else -1
            pA = 1 if abs(m - 1) % 2 == 0 else -1
            odd = (pA if POLAR[c] else pS) == -1
            want = want + np.real((rp if odd else 1.0) * (F[c, 0] + F[c, 1] * zp / 5) * np.exp(1j * m * th))
        assert np.max(np.abs(got[:, c] - want)) < 1e-11 * max(1.0, np.max(np.abs(want))), (order, ss, c)


@pytest.mark.parametrize("ss", [1, 2, 3])
def test_supersampling_quarters_the_shape_smoothing(ss):
    """E_z of mode 0 (z staggered, rho primary, even) set to cos(kz z) cos(kr rho) on its own positions,
    every other component 0; kz dz = kr drho = 0.1, order 16 (the half shifts are exact to ~1e-20)."""
    g = grid(0, 16, nz=120, nr=40)
    kz, kr = 0.1 / g.dz, 0.1 / g.dr
    z = (np.arange(g.nz) - 0.5) * g.dz
    r = (np.arange(g.nr) + 0.5) * g.dr
    psi = np.zeros((6, g.nr, g.nz), complex)
    psi[2] = np.cos(kr * r)[:, None] * np.cos(kz * z)[None, :]
    rng = np.random.default_rng(ss)
    s = samples(rng, 300, g, 12, (g.nr - 12) * g.dr)
    zp, rp = s[:, 0], np.hypot(s[:, 1], s[:, 2])
    f = np.cos(kz * zp) * np.cos(kr * rp)
    err_plain = oracle.gather_fine([g], [psi], s, 0)[:, 2] - f
    err_fine = oracle.gather_fine([g], [psi], s, ss)[:, 2] - f
    # leading smoothing error (h^2/6) f'' per direction, h halved in the doubled directions
    hz2 = g.dz ** 2 / (4.0 if ss & 1 else 1.0)
    hr2 = g.dr ** 2 / (4.0 if ss & 2 else 1.0)
    pred_plain = -(kz ** 2 * g.dz ** 2 + kr ** 2 * g.dr ** 2) / 6 * f
    pred_fine = -(kz ** 2 * hz2 + kr ** 2 * hr2) / 6 * f
    scale = np.max(np.abs(pred_fine))
    assert np.max(np.abs(err_plain - pred_plain)) < 0.02 * np.max(np.abs(pred_plain))
    assert np.max(np.abs(err_fine - pred_fine)) < 0.02 * scale, (np.max(np.abs(err_fine - pred_fine)), scale)


def table1():
    """Rows of the paper's Table 1 (tests/golden): component -> (rho stagger, z stagger, symmetry, q for
    m = 0, 1, 2)."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_staggering_symmetry.txt")
    rows = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, sr, sz, sym, *q = line.split()
        rows[name] = (Fraction(sr), Fraction(sz), sym, [int(v) for v in q])
    return rows


def test_component_layout_matches_table1():
    """The staggering and symmetry types the interpolation tests (and the GPU gather tests that import
    them) assume are the printed ones, and the printed exponents are |m - 1| (mA) or m (mS)."""
    t = table1()
    names = ["E_rho", "E_theta", "E_z", "B_rho", "B_theta", "B_z"]
    for c, name in enumerate(names):
        sr, sz, sym, q = t[name]
        assert RST[c] == (sr != 0) and ZST[c] == (sz != 0), name
        assert POLAR[c] == (sym == "mA"), name
        assert q == [abs(m - 1) if sym == "mA" else m for m in range(3)], name


@pytest.mark.parametrize("m", [0, 1, 2])
def test_half_shifts_follow_table1_near_the_axis(m):
    """For each component and m = 0, 1, 2, a field rho^q (1 + (rho/4)^2) with q from Table 1, sampled on
    the component's rho positions, is shifted exactly by the oracle's half shift towards the other rho
    positions on every row next to the axis: S^(+) with the component's parity and axis rule (extrapolate
    exactly when the table says constant on the axis) for staggered components, S^(-) on rows k >= 1 for
    primary ones.  Order 8."""
    t = table1()
    g = grid(m, 8)
    pS = 1 if m % 2 == 0 else -1
    pA = 1 if abs(m - 1) % 2 == 0 else -1
    r_st = np.arange(g.nr) * g.dr
    r_pr = (np.arange(g.nr) + 0.5) * g.dr
    rows = slice(0, g.nr - 4)
    for name, (sr, _, sym, qs) in t.items():
        if name == "phi":
            continue
        q = qs[m]
        f = lambda r: r ** q * (1.0 + (r / 4) ** 2)
        parity = pA if sym == "mA" else pS
        if sr != 0:  # stored on the staggered rows: S^(+) to the primary rows
            plane = np.repeat(f(r_st)[:, None], g.nz, 1).astype(complex)
            plane[0] = 77.0  # axis slot: derived, never read
            out = oracle.apply_op(g, oracle.OP_SHIFT_PLUS_RHO, plane, parity, q == 0)
            want = f(r_pr)
        else:  # stored on the primary rows: S^(-) to the staggered rows k >= 1
            plane = np.repeat(f(r_pr)[:, None], g.nz, 1).astype(complex)
            out = oracle.apply_op(g, oracle.OP_SHIFT_MINUS, plane, parity)
            want = f(r_st)
            out, want = out[1:], want[1:]
        err = np.max(np.abs(out[rows] - want[rows, None]))
        assert err < 1e-12 * max(1.0, np.max(np.abs(want))), (name, m, err)
