"""GPU deposition of point samples into J_z (fdetd_deposit_jz) and the charge density (fdetd_deposit_rho)
against the oracle's deposition, and the discrete continuity equation between the GPU's own outputs.

A bunch of samples concentrated near the axis (the shapes fold across it there) plus a spread of samples,
including some within two cells of the z ends (skipped by both sides), is deposited for modes 0, 1, 2 of
one grid in one batched plan.  The adds are atomic, so only the order of the summation differs from the
oracle: FP64 agrees to relative L2 <= 1e-12 per mode.  FP32C adds values formed in FP64 with float atomics
in a varying order: each add rounds the running sum (float epsilon 6e-8), a cell takes a few hundred adds
of random-sign weights whose partial sums exceed the final value several times, so the bound is 1e-5
(runs measure 5e-7 .. 1.3e-6).  The deposit adds into plane 2 only.
"""
import math

import numpy as np
import pytest

from helpers import dev, log, rel_l2

import oracle
import paper_2605_12132_amd as F
import paper_2605_12132_amd.inputs as I

pytestmark = pytest.mark.gpu


def samples(rng, n, nz, nr, dz, dr):
    z = np.concatenate([rng.normal(0.4 * nz * dz, 6 * dz, n // 2), rng.uniform(0, nz * dz, n - n // 2)])
    r = np.concatenate([np.abs(rng.normal(0, 2.0 * dr, n // 2)), rng.uniform(0, nr * dr, n - n // 2)])
    th = rng.uniform(-math.pi, math.pi, n)
    w = rng.uniform(-1.0, 1.0, n) * 1e-2
    return np.stack([z, r * np.cos(th), r * np.sin(th), w], axis=1)


@pytest.mark.parametrize("precision", [0, 1])
def test_deposit_matches_oracle(precision):
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr = 300, 48
    w = I.Workload("dep", 0, [nz] * 3, [nr] * 3, [0, 1, 2], [16] * 3, 8, dz, 2 * dz, 0.5 * dz, 1)
    rng = np.random.default_rng(21)
    s = samples(rng, 20000, nz, nr, dz, 2 * dz)
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=1)
    base = [0.01 * (rng.uniform(-1, 1, (3, nr, nz)) + 1j * rng.uniform(-1, 1, (3, nr, nz))) for _ in range(3)]
    J = [dev(b, cd) for b in base]
    plan.deposit_jz(dev(s, torch.float64), J, vz=1.0, eps=0.5)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == F.FP64 else 1e-5
    for p in range(3):
        g = oracle.Grid(nz=nz, nr=nr, m=p, fd_order=16, taylor_order=8, dz=dz, dr=2 * dz, dt=0.5 * dz)
        want = oracle.deposit_jz(g, s, vz=1.0, eps=0.5)
        got = J[p].cpu().numpy().astype(np.complex128) - base[p]
        err = rel_l2(got[2], want[2])
        log(f"deposit m={p} precision={precision}: rel L2 {err:.2e}")
        assert err < tol
        assert np.max(np.abs(got[:2])) < 1e-15 if precision == F.FP64 else np.max(np.abs(got[:2])) < 1e-8
    plan.close()


def test_deposit_rejects_bad_arguments():
    import torch
    dz = I.LAMBDA0 / 20
    w = I.Workload("dep", 0, [64], [16], [0], [8], 8, dz, 2 * dz, 0.5 * dz, 1)
    plan = F.Plan(w.problems(), precision=F.FP64, flags=1)
    J = [torch.zeros((3, 16, 64), dtype=torch.complex128, device="cuda")]
    s = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    for kw in (dict(vz=float("inf")), dict(vz=float("nan")), dict(eps=1.5)):
        with pytest.raises(F.FdetdError):
            plan.deposit_jz(s, J, **kw)
    plan.deposit_jz(s[:0], J)  # no samples: nothing to do
    torch.cuda.synchronize()
    assert torch.count_nonzero(J[0]) == 0
    plan.close()


@pytest.mark.parametrize("ordered", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
def test_deposit_rho_matches_oracle_and_continuity(precision, ordered):
    """Charge densities of the samples shifted by -+ vz dt/2 against the oracle (same tolerances as J_z),
    and, FP64, the discrete continuity equation between the GPU's two densities and its J_z:
    (rho_+(i) - rho_-(i)) / dt + (J_z(i + 1/2) - J_z(i - 1/2)) / dz = 0 to rounding.  Samples in z order
    go through the LDS tiles, unordered ones through global atomics."""
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr = 260, 40
    dt = 0.5 * dz
    w = I.Workload("dep", 0, [nz] * 3, [nr] * 3, [0, 1, 2], [8] * 3, 8, dz, 2 * dz, dt, 1)
    rng = np.random.default_rng(33)
    s = samples(rng, 12000, nz, nr, dz, 2 * dz)
    if ordered:
        s = s[np.argsort(s[:, 0], kind="stable")]
    sd = dev(s, torch.float64)
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=1)
    vz = 0.9
    rp = [torch.zeros((nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    rm = [torch.zeros((nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    J = [torch.zeros((3, nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    plan.deposit_rho(sd, rp, dz_shift=0.5 * vz * dt, eps=0.5)
    plan.deposit_rho(sd, rm, dz_shift=-0.5 * vz * dt, eps=0.5)
    plan.deposit_jz(sd, J, vz=vz, eps=0.5)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == F.FP64 else 1e-5
    for p in range(3):
        g = oracle.Grid(nz=nz, nr=nr, m=p, fd_order=8, taylor_order=8, dz=dz, dr=2 * dz, dt=dt)
        want = oracle.deposit_rho(g, s, 0.5 * vz * dt, eps=0.5)
        got = rp[p].cpu().numpy().astype(np.complex128)
        err = rel_l2(got, want)
        log(f"deposit rho m={p} precision={precision} ordered={ordered}: rel L2 {err:.2e}")
        assert err < tol
        if precision == F.FP64:
            # samples skipped by the current (shape past a z end at either position) are also skipped by
            # one of the densities; compare on columns away from the ends, where nothing is skipped
            a = rp[p].cpu().numpy()
            b = rm[p].cpu().numpy()
            jz = J[p][2].cpu().numpy()
            res = (a - b)[:, 8:nz - 8] / dt + (jz[:, 9:nz - 7] - jz[:, 8:nz - 8]) / dz
            scale = np.max(np.abs(a)) / dt
            log(f"  continuity residual {np.max(np.abs(res)) / scale:.2e} of max |rho| / dt")
            assert np.max(np.abs(res)) < 1e-12 * scale
    with pytest.raises(F.FdetdError):
        plan.deposit_rho(sd, rp, eps=2.0)
    plan.close()


def moving_samples(rng, n, nz, nr, dz, dr, dt):
    s = samples(rng, n, nz, nr, dz, dr)
    v = rng.uniform(-0.8, 0.8, (n, 3))
    return np.column_stack([s, v, np.zeros(n)])


@pytest.mark.parametrize("ordered", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
def test_deposit_current_of_moving_samples(precision, ordered):
    """All four planes (J_rho, J_theta, J_z, rho_xy) of moving samples against the oracle, modes 0..2 in
    one plan with the current correction (FP64 1e-12, FP32C 1e-5 as for J_z), and, FP64, the split of the
    continuity equation between the GPU's own J_z and rho_xy and the oracle's densities at the end
    positions."""
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr, dt = 200, 36, 0.5 * dz
    w = I.Workload("dep", 0, [nz] * 3, [nr] * 3, [0, 1, 2], [8] * 3, 8, dz, 2 * dz, dt, 1)
    rng = np.random.default_rng(44)
    s = moving_samples(rng, 8000, nz, nr, dz, 2 * dz, dt)
    if ordered:  # z order: blocks accumulate in LDS tiles
        s = s[np.argsort(s[:, 0], kind="stable")]
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=1 | F.PLAN_CURRENT_CORRECTION)
    J = [torch.zeros((4, nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    plan.deposit_current(dev(s, torch.float64), J, eps=0.5)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == F.FP64 else 1e-5
    for p in range(3):
        g = oracle.Grid(nz=nz, nr=nr, m=p, fd_order=8, taylor_order=8, dz=dz, dr=2 * dz, dt=dt)
        wj, wr = oracle.deposit_current(g, s)
        got = J[p].cpu().numpy().astype(np.complex128)
        errs = [rel_l2(got[c], wj[c]) for c in range(3)] + [rel_l2(got[3], wr)]
        log(f"deposit current m={p} precision={precision} ordered={ordered}: rel L2 per plane "
            f"{[f'{e:.1e}' for e in errs]}")
        assert max(errs) < tol
        if precision == F.FP64:
            h = 0.5 * dt
            plus, minus = s[:, :4].copy(), s[:, :4].copy()
            plus[:, :3] += h * s[:, [6, 4, 5]]
            minus[:, :3] -= h * s[:, [6, 4, 5]]
            rp, rm = oracle.deposit_rho(g, plus), oracle.deposit_rho(g, minus)
            res = (rp - rm)[:, 8:nz - 8] / dt + (got[2][:, 9:nz - 7] - got[2][:, 8:nz - 8]) / dz - got[3][:, 8:nz - 8]
            assert np.max(np.abs(res)) < 1e-11 * np.max(np.abs(got[3]))
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_deposit_jz_position_ordered_samples(precision):
    """Samples sorted by z: the blocks' footprints are small, so the deposition accumulates them in LDS
    tiles before adding to the grid; the result matches the oracle to the same tolerances."""
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr = 400, 64
    w = I.Workload("dep", 0, [nz] * 3, [nr] * 3, [0, 1, 2], [16] * 3, 8, dz, 2 * dz, 0.5 * dz, 1)
    rng = np.random.default_rng(8)
    s = samples(rng, 30000, nz, nr, dz, 2 * dz)
    s = s[np.argsort(s[:, 0], kind="stable")]
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=1)
    J = [torch.zeros((3, nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    plan.deposit_jz(dev(s, torch.float64), J, vz=1.0, eps=0.5)
    torch.cuda.synchronize()
    tol = 1e-12 if precision == F.FP64 else 1e-5
    for p in range(3):
        g = oracle.Grid(nz=nz, nr=nr, m=p, fd_order=16, taylor_order=8, dz=dz, dr=2 * dz, dt=0.5 * dz)
        want = oracle.deposit_jz(g, s, vz=1.0, eps=0.5)
        err = rel_l2(J[p].cpu().numpy().astype(np.complex128)[2], want[2])
        log(f"ordered deposit m={p} precision={precision}: rel L2 {err:.2e}")
        assert err < tol
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_samples_on_the_axis_deposit_only_into_mode_0(precision):
    """Section 3.5 folds the shape below the axis antisymmetrically for m > 1 (m_S / m_A type for m <= 1):
    samples on the axis deposit nothing into modes 1..4, through every deposition kernel; mode 0 gets it."""
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr = 120, 24
    modes = [0, 1, 2, 3, 4]
    w = I.Workload("axis", 0, [nz] * 5, [nr] * 5, modes, [8] * 5, 8, dz, 2 * dz, 0.5 * dz, 1)
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY | F.PLAN_CURRENT_CORRECTION)
    z = np.linspace(40 * dz, 80 * dz, 64)
    s4 = np.stack([z, np.zeros(64), np.zeros(64), np.ones(64)], axis=1)
    s8 = np.column_stack([s4, np.zeros((64, 2)), np.full(64, 0.9), np.zeros(64)])
    J3 = [torch.zeros((3, nr, nz), dtype=cd, device="cuda") for _ in modes]
    J4 = [torch.zeros((4, nr, nz), dtype=cd, device="cuda") for _ in modes]
    R1 = [torch.zeros((nr, nz), dtype=cd, device="cuda") for _ in modes]
    plan.deposit_jz(dev(s4, torch.float64), J3, vz=0.9, eps=0.5)
    plan.deposit_current(dev(s8, torch.float64), J4, eps=0.5)
    plan.deposit_rho(dev(s4, torch.float64), R1, eps=0.5)
    torch.cuda.synchronize()
    for p, m in enumerate(modes):
        peak = max(float(torch.max(torch.abs(x[p]))) for x in (J3, J4, R1))
        if m == 0:
            assert peak > 0
        else:
            assert peak == 0.0, (m, peak)
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_fast_samples_deposit_their_whole_shape(precision):
    """Samples that move 3 to 9 cells in a step (integrated z shapes over more than 8 nodes) take the
    kernels' global-atomic path; J_z of fdetd_deposit_jz (uniform vz) and all currents and rho_xy of
    fdetd_deposit_current (per-sample velocities, mixed with slow ones in the same blocks) equal the
    oracle's (tolerances as above)."""
    import torch
    dz = I.LAMBDA0 / 20
    nz, nr = 200, 24
    w = I.Workload("fast", 0, [nz] * 3, [nr] * 3, [0, 1, 2], [8] * 3, 8, dz, 2 * dz, 0.5 * dz, 1)
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    tol = 1e-12 if precision == F.FP64 else 1e-5
    rng = np.random.default_rng(33)
    n = 3000
    z = rng.uniform(14 * dz, (nz - 15) * dz, n)
    r = np.abs(rng.normal(0, 4 * dz, n))
    th = rng.uniform(-math.pi, math.pi, n)
    s4 = np.stack([z, r * np.cos(th), r * np.sin(th), rng.uniform(-1, 1, n) * 1e-2], axis=1)
    plan0 = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY)
    plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY | F.PLAN_CURRENT_CORRECTION)
    vz = 13.0  # 6.5 cells per step
    J = [torch.zeros((3, nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    plan0.deposit_jz(dev(s4, torch.float64), J, vz=vz, eps=0.5)
    s8 = np.zeros((n, 8))
    s8[:, :4] = s4
    s8[:, 4:6] = rng.uniform(-0.3, 0.3, (n, 2))
    s8[:, 6] = rng.choice([-1.0, 1.0], n) * np.where(rng.uniform(0, 1, n) < 0.5, rng.uniform(6.5, 18.0, n),
                                                     rng.uniform(0.0, 0.9, n))
    J8 = [torch.zeros((4, nr, nz), dtype=cd, device="cuda") for _ in range(3)]
    plan.deposit_current(dev(s8, torch.float64), J8, eps=0.5)
    torch.cuda.synchronize()
    for p in range(3):
        g = oracle.Grid(nz=nz, nr=nr, m=p, fd_order=8, taylor_order=8, dz=dz, dr=2 * dz, dt=0.5 * dz)
        want = oracle.deposit_jz(g, s4, vz=vz, eps=0.5)
        got = J[p].cpu().numpy().astype(np.complex128)
        e1 = rel_l2(got[2], want[2])
        wj, wr = oracle.deposit_current(g, s8, eps=0.5)
        got8 = J8[p].cpu().numpy().astype(np.complex128)
        e2 = max(rel_l2(got8[c], wj[c]) for c in range(3))
        e3 = rel_l2(got8[3], wr)
        log(f"fast samples m={p} precision={precision}: J_z {e1:.2e}, currents {e2:.2e}, rho_xy {e3:.2e}")
        assert np.max(np.abs(want[2])) > 0 and e1 < tol and e2 < tol and e3 < tol
    plan.close()
    plan0.close()
