"""Pins of the oracle's deposition of moving samples (section 3.6, with the planar density differential of
section 3.7):

* samples moving along z only reproduce the longitudinal current of oracle.deposit_jz and deposit no
  transverse current and no planar density differential;
* the charge densities of the samples at their end positions (x, y, z) +- v dt/2, deposited with
  oracle.deposit_rho, satisfy  (rho+ - rho-)/dt + D_z^(+) J_z - rho_xy = 0  exactly: the z current takes
  the longitudinal change and rho_xy the transverse one (the split of section 3.7);
* away from the axis J_rho and J_theta are the sample's v_rho and v_theta times its density shape;
* next to the axis, a uniform density drifting along x gives the m = 1 mode J_rho = n q v, J_theta = i n q v
  on every row (the m_A fold of the radial shape), and no m = 0 or m = 2 current.
"""
import math

import numpy as np

import oracle


def grid(m, nz=40, nr=16):
    return oracle.Grid(nz=nz, nr=nr, m=m, fd_order=8, taylor_order=4, dz=0.3, dr=0.4, dt=0.15)


def moving(rng, n, g, vmax=0.6, rmax=None):
    rmax = rmax if rmax is not None else (g.nr - 3) * g.dr
    z = rng.uniform(4 * g.dz, (g.nz - 5) * g.dz, n)
    r = np.sqrt(rng.uniform(0, rmax ** 2, n))
    th = rng.uniform(-math.pi, math.pi, n)
    v = rng.uniform(-vmax, vmax, (n, 3))
    return np.column_stack([z, r * np.cos(th), r * np.sin(th), rng.uniform(-1, 1, n), v, np.zeros(n)])


def test_longitudinal_motion_reduces_to_deposit_jz():
    rng = np.random.default_rng(1)
    for m in (0, 1, 2):
        g = grid(m)
        s = moving(rng, 300, g)
        s[:, 4:6] = 0.0
        s[:, 6] = 0.7
        j, rxy = oracle.deposit_current(g, s)
        want = oracle.deposit_jz(g, s[:, :4], vz=0.7)
        assert np.max(np.abs(j[2] - want[2])) < 1e-13 * np.max(np.abs(want[2]))
        assert not np.any(j[:2]) and not np.any(rxy)


def test_continuity_splits_into_longitudinal_and_planar_parts():
    rng = np.random.default_rng(2)
    for m in (0, 1, 3):
        g = grid(m)
        s = moving(rng, 400, g)
        j, rxy = oracle.deposit_current(g, s)
        h = 0.5 * g.dt
        plus, minus = s[:, :4].copy(), s[:, :4].copy()
        plus[:, :3] += h * s[:, [6, 4, 5]]
        minus[:, :3] -= h * s[:, [6, 4, 5]]
        rp, rm = oracle.deposit_rho(g, plus), oracle.deposit_rho(g, minus)
        # D_z^(+) of the staggered J_z (J_z(i - 1/2) stored at column i) at primary column i
        dzj = np.zeros_like(j[2])
        dzj[:, :-1] = (j[2][:, 1:] - j[2][:, :-1]) / g.dz
        res = (rp - rm) / g.dt + dzj - rxy
        cols = slice(2, g.nz - 3)
        assert np.max(np.abs(res[:, cols])) < 1e-12 * np.max(np.abs(rxy)), m


def test_transverse_currents_away_from_axis():
    rng = np.random.default_rng(3)
    for m in (0, 1, 2):
        g = grid(m, nr=24)
        s = moving(rng, 50, g, rmax=(g.nr - 4) * g.dr)
        r = np.hypot(s[:, 1], s[:, 2])
        s = s[r > 5 * g.dr]  # shapes that do not reach the axis
        r = np.hypot(s[:, 1], s[:, 2])
        vr = (s[:, 1] * s[:, 4] + s[:, 2] * s[:, 5]) / r
        vt = (s[:, 1] * s[:, 5] - s[:, 2] * s[:, 4]) / r
        j, _ = oracle.deposit_current(g, s)
        wr, wt = s[:, :4].copy(), s[:, :4].copy()
        wr[:, 3] *= vr
        wt[:, 3] *= vt
        assert np.max(np.abs(j[0] - oracle.deposit_rho(g, wr))) < 1e-13 * np.max(np.abs(j[0]))
        assert np.max(np.abs(j[1] - oracle.deposit_rho(g, wt))) < 1e-13 * np.max(np.abs(j[1]))


def test_uniform_drift_next_to_axis():
    """Samples on a fine Cartesian lattice filling a disk (unit charge density), all moving with v_x."""
    g1, g0, g2 = grid(1, nz=24), grid(0, nz=24), grid(2, nz=24)
    h, R, v = g1.dr / 4, 8 * g1.dr, 0.3
    xs = np.arange(-R, R, h) + h / 2
    X, Y = np.meshgrid(xs, xs)
    keep = X ** 2 + Y ** 2 < R ** 2
    X, Y = X[keep], Y[keep]
    zs = np.arange(8 * g1.dz, 16 * g1.dz, g1.dz / 2) + g1.dz / 4
    n = X.size * zs.size
    s = np.column_stack([np.repeat(zs, X.size), np.tile(X, zs.size), np.tile(Y, zs.size),
                         np.full(n, h * h * g1.dz / 2), np.full(n, v), np.zeros(n), np.zeros(n), np.zeros(n)])
    j1, _ = oracle.deposit_current(g1, s)
    i = 12
    rows = slice(0, 5)  # next to the axis, inside the disk by more than the shape width
    assert np.max(np.abs(j1[0, rows, i] - v)) < 5e-3 * v
    assert np.max(np.abs(j1[1, rows, i] - 1j * v)) < 5e-3 * v
    for g in (g0, g2):
        j, _ = oracle.deposit_current(g, s)
        assert np.max(np.abs(j[:2, rows, i])) < 1e-3 * v


def test_fast_samples_keep_the_whole_integrated_shape():
    """Samples that move 3 to 9 cells along z in one step (large dt or |v| > c): the integrated shape of
    section 3.6 spans every node between the two positions, so the continuity equation still holds exactly
    and the z current integrates to q w v_z times the (radial, angular) shape, i.e. the charge moved per
    unit time."""
    rng = np.random.default_rng(5)
    for m in (0, 1, 2):
        g = oracle.Grid(nz=60, nr=16, m=m, fd_order=8, taylor_order=4, dz=0.3, dr=0.4, dt=0.15)
        s = moving(rng, 200, g)
        s[:, 0] = rng.uniform(12 * g.dz, (g.nz - 13) * g.dz, s.shape[0])
        s[:, 6] = rng.choice([-1.0, 1.0], s.shape[0]) * rng.uniform(6.0, 18.0, s.shape[0])  # 3 .. 9 cells
        assert np.min(np.abs(s[:, 6])) * g.dt / g.dz > 3.0
        j, rxy = oracle.deposit_current(g, s)
        h = 0.5 * g.dt
        plus, minus = s[:, :4].copy(), s[:, :4].copy()
        plus[:, :3] += h * s[:, [6, 4, 5]]
        minus[:, :3] -= h * s[:, [6, 4, 5]]
        rp, rm = oracle.deposit_rho(g, plus), oracle.deposit_rho(g, minus)
        dzj = np.zeros_like(j[2])
        dzj[:, :-1] = (j[2][:, 1:] - j[2][:, :-1]) / g.dz
        res = (rp - rm) / g.dt + dzj - rxy
        assert np.max(np.abs(res[:, 2:g.nz - 3])) < 1e-12 * np.max(np.abs(rp - rm) / g.dt), m
        # one sample: sum_i J_z dz = q w v_z * (mean of the two end-position shapes) on every row
        one = s[:1].copy()
        one[0, 4:6] = 0.0
        j1, _ = oracle.deposit_current(g, one)
        shape = oracle.deposit_rho(g, one[:, :4]).sum(axis=1) * g.dz  # q w R_k A_m
        assert np.max(np.abs(j1[2].sum(axis=1) * g.dz - one[0, 6] * shape)) < 1e-12 * np.max(np.abs(one[0, 6] * shape))
