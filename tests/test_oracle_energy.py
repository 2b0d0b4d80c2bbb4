"""Pins of the oracle's energy diagnostics (section 5.1, eqs. test_am_vacuum_E and test_am_vacuum_Z):
<E> = integral of |E|^2 + |B|^2 over the volume, <z> its first moment over <E>; for the envelope the
integrand is |a~ - i k0 a|^2 (eq. laserA_envelope_E).

* Parseval: the oracle's energy of one mode equals the energy of the real 3D field Re(F_m e^(i m theta))
  integrated over theta on a theta grid (the trapezoid rule is exact for these trigonometric polynomials).
  A wrong mode weight (pi against 2 pi) fails.
* Analytic volume integrals: components of the form rho exp(-rho^2/s^2) exp(-(z - z0)^2/L^2), sampled at
  their own staggered positions (Table 1), have the closed-form energy (2 pi or pi) (s^2/2)^2 / 2 L sqrt(pi/2)
  per component, and centroid z0.  Radial weights of the wrong grid (rho_k for a rho-staggered component),
  or z positions of the wrong grid, fail.
"""
import math

import numpy as np
import pytest

import oracle

# rho-staggered and z-staggered flags of E_rho, E_theta, E_z, B_rho, B_theta, B_z (Table 1)
RST = [1, 0, 0, 0, 1, 1]
ZST = [0, 0, 1, 1, 1, 0]


def positions(g, c):
    r = np.arange(g.nr) * g.dr if RST[c] else (np.arange(g.nr) + 0.5) * g.dr
    z = (np.arange(g.nz) - 0.5) * g.dz if ZST[c] else np.arange(g.nz) * g.dz
    return r, z


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_energy_is_the_theta_integral_of_the_real_field(m):
    g = oracle.Grid(nz=20, nr=10, m=m, fd_order=4, taylor_order=4, dz=0.3, dr=0.4, dt=0.1)
    rng = np.random.default_rng(40 + m)
    psi = rng.uniform(-1, 1, (6, g.nr, g.nz)) + 1j * rng.uniform(-1, 1, (6, g.nr, g.nz))
    if m == 0:
        psi = psi.real.astype(complex)  # the m = 0 mode is real (its imaginary part is discarded)
    nth = 16
    th = 2 * math.pi * np.arange(nth) / nth
    W3 = Wz3 = 0.0
    for c in range(6):
        r, z = positions(g, c)
        f = (psi[c][None] * np.exp(1j * m * th)[:, None, None]).real  # [theta, rho, z]
        dens = np.sum(f ** 2, axis=0) * (2 * math.pi / nth)          # integral over theta
        vol = r[:, None] * g.dr * g.dz
        W3 += np.sum(dens * vol)
        Wz3 += np.sum(dens * vol * z[None, :])
    W, zc = oracle.energy(g, psi)
    assert abs(W / W3 - 1) < 1e-13
    assert abs(zc - Wz3 / W3) < 1e-12 * g.nz * g.dz


@pytest.mark.parametrize("m", [0, 1, 2])
def test_energy_and_centroid_of_analytic_fields(m):
    s, L, z0 = 3.2, 2.5, 10.0
    g = oracle.Grid(nz=200, nr=64, m=m, fd_order=4, taylor_order=4, dz=0.1, dr=0.2, dt=0.05)
    psi = np.zeros((6, g.nr, g.nz), complex)
    amp = [1.0, 0.5j, -0.7, 0.3 + 0.4j, 1.1, -0.2j]
    for c in range(6):
        r, z = positions(g, c)
        psi[c] = amp[c] * (r * np.exp(-(r / s) ** 2))[:, None] * np.exp(-((z - z0) / L) ** 2)[None, :]
    if m == 0:
        psi = np.abs(psi).astype(complex)
    wm = 2 * math.pi if m == 0 else math.pi
    per = wm * 0.5 * (s * s / 2) ** 2 * L * math.sqrt(math.pi / 2)  # one component of unit amplitude
    want = per * sum(abs(a) ** 2 for a in amp)
    W, zc = oracle.energy(g, psi)
    assert abs(W / want - 1) < 1e-6, (W, want)
    assert abs(zc - z0) < 1e-9 * L, (zc, z0)


def test_envelope_energy_of_analytic_fields():
    """|a~ - i k0 a|^2 with a~ = 0 gives k0^2 |a|^2; with a = 0 it gives |a~|^2; both integrate in closed form
    (m = 0 weight 2 pi, primary positions)."""
    s, L, z0, k0 = 3.2, 2.5, 10.0, 1.7
    g = oracle.Grid(nz=200, nr=64, m=0, fd_order=4, taylor_order=4, dz=0.1, dr=0.2, dt=0.05, k0=k0)
    r = (np.arange(g.nr) + 0.5) * g.dr
    z = np.arange(g.nz) * g.dz
    f = (r * np.exp(-(r / s) ** 2))[:, None] * np.exp(-((z - z0) / L) ** 2)[None, :]
    unit = 2 * math.pi * 0.5 * (s * s / 2) ** 2 * L * math.sqrt(math.pi / 2)
    W, zc = oracle.envelope_energy(g, (0.6 - 0.8j) * f, np.zeros_like(f, complex))
    assert abs(W / (k0 ** 2 * unit) - 1) < 1e-6 and abs(zc - z0) < 1e-9 * L
    W, zc = oracle.envelope_energy(g, np.zeros_like(f, complex), 2.0j * f)
    assert abs(W / (4 * unit) - 1) < 1e-6 and abs(zc - z0) < 1e-9 * L
    # a~ = i k0 a cancels: the field envelope vanishes
    W, _ = oracle.envelope_energy(g, f.astype(complex), 1j * k0 * f)
    assert W < 1e-28
