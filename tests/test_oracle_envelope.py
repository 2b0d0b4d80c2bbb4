"""Pins of the oracle's laser-envelope operator H_a and its exponential step (section 4).

* Bessel modes a = J_m(g rho) exp(i k z) satisfy (grad^2_perp,m + dz^2) a = -(g^2 + k^2) a, dz a = i k a:
  the discrete H_a of section 4.2 (L_rho + L_z - m^2/rho^2, D_z^(C), mS symmetry) must converge to it.
* For m = 0 fields uniform in rho and uniform chi, each z-Fourier mode evolves by the 2x2 matrix
  [[0, 1], [-k2 - chi - 2 k0 k1, 2 i k0]] (k1, k2: symbols of D_z^(C), -L_z); after K steps the interior
  equals T_N(dt A)^K exactly.
* On tiny grids the step equals the dense matrix exponential within the Taylor remainder bound.
* Reading of the printed real 4x4 operator: applied to (Re, Im) of the conjugate state it gives the
  conjugate of the complex equation -- it propagates the conjugate envelope.
* Physics: a Gaussian envelope in uniform plasma moves at (c - v_g)/c = n0/(2 n_c) + (lambda/(2 pi w0))^2.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.special import jv

import oracle


def bessel_env_residual(m, order, scale, near_axis, chi0=0.3, k0=1.0):
    nd = order // 2
    nr, nz = int(24 * scale) + nd, int(24 * scale) + 2 * nd
    g = oracle.Grid(nz=nz, nr=nr, m=m, fd_order=order, taylor_order=1, dz=0.25 / scale, dr=0.3 / scale,
                    dt=0.0, k0=k0)
    gam, kz = 1.3, 1.1
    rho = (np.arange(nr) + 0.5) * g.dr
    z = np.arange(nz) * g.dz
    a = jv(m, gam * rho)[:, None] * np.exp(1j * kz * z)[None, :]
    at = (0.3 - 0.7j) * a
    chi = np.full((nr, nz), chi0)
    oa, ot = oracle.apply_Ha(g, a, at, chi)
    want = (-gam ** 2 - kz ** 2 - chi0 - 2 * k0 * kz) * a + 2j * k0 * at
    assert np.array_equal(oa, at)
    idx = np.arange(nr)
    rows = idx[:nd + 1] if near_axis else idx[(rho >= 1.5) & (idx < nr - nd)]
    return np.max(np.abs(ot[rows][:, nd:nz - nd] - want[rows][:, nd:nz - nd]))


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_envelope_bessel_modes_converge(m, order):
    e1, e2 = bessel_env_residual(m, order, 2, False), bessel_env_residual(m, order, 4, False)
    assert math.log2(e1 / e2) > order - 0.2, (e1, e2)
    e1, e2 = bessel_env_residual(m, order, 2, True), bessel_env_residual(m, order, 4, True)
    assert math.log2(e1 / e2) > order - 1.1, (e1, e2)


def taylor(x, N):
    return sum(np.linalg.matrix_power(x, n) / math.factorial(n) for n in range(N + 1))


@pytest.mark.parametrize("order,N,K", [(8, 4, 3), (4, 8, 2)])
def test_envelope_closed_form_per_mode(order, N, K):
    nd = order // 2
    reach = K * N * nd
    nz, nr = 2 * reach + 40, reach + 10
    g = oracle.Grid(nz=nz, nr=nr, m=0, fd_order=order, taylor_order=N, dz=0.4, dr=0.5, dt=0.2, k0=1.0)
    d = oracle.coef("d1", nd)
    b = oracle.coef("d2", nd)
    chi0 = 0.05
    kz = 2 * np.pi / (9 * g.dz)
    k1 = 2 * sum(d[j] * np.sin((j + 1) * kz * g.dz) for j in range(nd)) / g.dz
    k2 = -(b[0] + 2 * sum(b[j] * np.cos(j * kz * g.dz) for j in range(1, nd + 1))) / g.dz ** 2
    A = np.array([[0, 1], [-k2 - chi0 - 2 * g.k0 * k1, 2j * g.k0]])
    T = np.linalg.matrix_power(taylor(g.dt * A, N), K)
    ph = np.exp(1j * kz * np.arange(nz) * g.dz)[None, :].repeat(nr, 0)
    a0, t0 = 1.0 + 0.5j, -0.3 + 0.2j
    a, at = oracle.envelope_step(g, a0 * ph, t0 * ph, np.full((nr, nz), chi0), K)
    wa, wt = T @ np.array([a0, t0])
    cols = slice(reach + 1, nz - reach - 1)
    rows = slice(0, nr - reach - 1)
    assert np.max(np.abs(a[rows, cols] - wa * ph[rows, cols])) < 1e-12
    assert np.max(np.abs(at[rows, cols] - wt * ph[rows, cols])) < 1e-12


def dense_Ha(g, chi):
    n = g.nr * g.nz
    H = np.zeros((2 * n, 2 * n), complex)
    e = np.zeros(2 * n, complex)
    for q in range(2 * n):
        e[q] = 1.0
        oa, ot = oracle.apply_Ha(g, e[:n].reshape(g.nr, g.nz), e[n:].reshape(g.nr, g.nz), chi)
        H[:n, q], H[n:, q] = oa.ravel(), ot.ravel()
        e[q] = 0.0
    return H


@pytest.mark.parametrize("m", [0, 2])
def test_envelope_step_equals_dense_expm(m):
    g = oracle.Grid(nz=12, nr=6, m=m, fd_order=4, taylor_order=6, dz=0.5, dr=0.6, dt=0.1, k0=1.0)
    rng = np.random.default_rng(21)
    chi = 0.01 * (1 + 0.05 * rng.uniform(-1, 1, (6, 12)))
    H = dense_Ha(g, chi)
    nrm = np.linalg.norm(H, 2)
    a = rng.standard_normal((6, 12)) + 1j * rng.standard_normal((6, 12))
    at = rng.standard_normal((6, 12)) + 1j * rng.standard_normal((6, 12))
    x = np.concatenate([a.ravel(), at.ravel()])
    for dt, N in ((0.1, 6), (0.05, 12), (0.2, 4)):
        g.dt, g.taylor_order = dt, N
        ga, gt = oracle.envelope_step(g, a, at, chi, 1)
        want = scipy.linalg.expm(dt * H) @ x
        got = np.concatenate([ga.ravel(), gt.ravel()])
        bound = sum((dt * nrm) ** n / math.factorial(n) for n in range(N + 1, N + 40)) * np.linalg.norm(x)
        assert np.linalg.norm(got - want) <= bound + 1e-13 * np.linalg.norm(x)


def test_printed_real_form_propagates_the_conjugate_envelope():
    g = oracle.Grid(nz=16, nr=8, m=0, fd_order=6, taylor_order=1, dz=0.5, dr=0.6, dt=0.0, k0=1.3)
    rng = np.random.default_rng(2)
    chi = rng.uniform(0, 0.1, (8, 16))
    a = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    at = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    lap = lambda f: (oracle.apply_op(g, oracle.OP_LAP_RHO, f.astype(complex), 1)
                     + oracle.apply_op(g, oracle.OP_LAP_Z, f.astype(complex))).real
    dzc = lambda f: oracle.apply_op(g, oracle.OP_DZ_CENTRED, f.astype(complex)).real
    # the 4x4 operator of section 4.2 on psi_a = (a_r, a_i, at_r, at_i), here fed the conjugate state
    ar, ai, tr, ti = a.real, -a.imag, at.real, -at.imag
    k0 = g.k0
    d_tr = lap(ar) - chi * ar + 2 * k0 * dzc(ai) + 2 * k0 * ti
    d_ti = -2 * k0 * dzc(ar) + lap(ai) - chi * ai - 2 * k0 * tr
    oa, ot = oracle.apply_Ha(g, a, at, chi)
    assert np.allclose(d_tr + 1j * d_ti, np.conj(ot), rtol=1e-12, atol=1e-12)
    assert np.allclose(tr + 1j * ti, np.conj(oa))


@pytest.mark.slow
def test_envelope_group_velocity_in_plasma_paper_case():
    """The plasma propagation test of section 5.2 with the paper's parameters: lambda = 0.8 um, n0 = 1e-3 n_c
    (chi = 1e-3), w0 = 16 um, field envelope length c tau = 10 um, 8th-order differences, 4th-order
    exponential, dt = dz / 2 with dz = lambda / 5.  The centroid of |a~ - i k0 a|^2, from its time derivative
    between t1 = T/10 and T, moves at (c - v_g)/c = n0/(2 n_c) + (lambda/(2 pi w0))^2 = 5.634e-4 (eq.
    test_am_plasma_vg), which the paper's envelope runs reproduce.  The formula is paraxial, not exact; its
    leading corrections here (finite bandwidth, O(chi^2)) are below 0.1 %.  Band: 2 %."""
    um = 2 * math.pi / 0.8
    k0, chi0, w0, L = 1.0, 1e-3, 16 * um, 10 * um
    dz, dr, T = 2 * math.pi / 5, 5.0, 600.0
    nr = int(math.ceil(2.6 * w0 / dr))                  # the beam's intensity is e^-13 at the outer edge
    zc = 3.2 * L
    nz = int(math.ceil((6.4 * L + T) / dz))
    g = oracle.Grid(nz=nz, nr=nr, m=0, fd_order=8, taylor_order=4, dz=dz, dr=dr, dt=0.5 * dz, k0=k0)
    z = np.arange(g.nz) * g.dz
    rho = (np.arange(g.nr) + 0.5) * g.dr
    a = np.exp(-(rho[:, None] / w0) ** 2 - ((z[None, :] - zc) / L) ** 2).astype(complex)
    # forward pulse: a~ = d a/dt ~ -v dz a - i (sqrt(k0^2 + chi) - k0) a
    om = math.sqrt(k0 ** 2 + chi0)
    at = -(k0 / om) * np.gradient(a, g.dz, axis=1) - 1j * (om - k0) * a
    chi = np.full((g.nr, g.nz), chi0)
    n1, n2 = int(round(0.1 * T / g.dt)), int(round(T / g.dt))
    a1, t1 = oracle.envelope_step(g, a, at, chi, n1)
    _, c1 = oracle.envelope_energy(g, a1, t1)
    a2, t2 = oracle.envelope_step(g, a1, t1, chi, n2 - n1)
    _, c2 = oracle.envelope_energy(g, a2, t2)
    delay = 1 - (c2 - c1) / ((n2 - n1) * g.dt)
    want = chi0 / 2 + (0.8 / (2 * math.pi * 16)) ** 2
    assert abs(want - 5.634e-4) < 1e-7
    assert abs(delay / want - 1) < 0.02, (delay, want)
