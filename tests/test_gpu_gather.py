"""GPU field interpolation at sample positions (fdetd_gather: destaggering, then cubic shapes over the
grid extended below the axis, summed over the modes; section 3.3) against the oracle, and against exact
values for states whose interpolation is exact.  FP64 to 1e-12 of the field scale; FP32C (destaggered
planes stored as floats) to 1e-5.  The same for 2x supersampling along z, rho and both
(fdetd_gather_supersampled, section 3.4) against the oracle's doubled-grid gather."""
import math

import numpy as np
import pytest

from helpers import dev, log

import oracle
import paper_2605_12132_amd as F
import paper_2605_12132_amd.inputs as I
from test_oracle_interpolation import POLAR, staggered_state

pytestmark = pytest.mark.gpu


def workload(modes, order, nz=150, nr=40, N=8):
    dz = I.LAMBDA0 / 20
    return I.Workload("gather", 0, [nz] * len(modes), [nr] * len(modes), list(modes), [order] * len(modes), N,
                      dz, 2 * dz, 0.5 * dz, 1)


def grids(w):
    return [oracle.Grid(nz=w.nz[p], nr=w.nr[p], m=w.m[p], fd_order=w.fd_order[p], taylor_order=w.taylor_order,
                        dz=w.dz, dr=w.dr, dt=w.dt) for p in range(w.n)]


def samples(rng, n, nz, nr, dz, dr):
    z = rng.uniform(-2 * dz, (nz + 1) * dz, n)  # some shapes reach past the z ends
    r = np.sqrt(rng.uniform(0, (nr + 1) ** 2, n)) * dr
    r[: n // 5] = rng.uniform(0, 2 * dr, n // 5)  # next to the axis
    th = rng.uniform(-math.pi, math.pi, n)
    return np.stack([z, r * np.cos(th), r * np.sin(th), np.ones(n)], axis=1)


def run(w, states, s, precision, supersample=0):
    import torch
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY)
    out = plan.gather([dev(x, cd) for x in states], dev(s, torch.float64), supersample=supersample)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    return got


@pytest.mark.parametrize("ordered", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("order", [8, 16])
def test_gather_matches_oracle(precision, order, ordered):
    w = workload([0, 1, 2], order)
    rng = np.random.default_rng(order + precision)
    states = [rng.uniform(-1, 1, (6, w.nr[0], w.nz[0])) + 1j * rng.uniform(-1, 1, (6, w.nr[0], w.nz[0]))
              for _ in range(w.n)]
    s = samples(rng, 5000, w.nz[0], w.nr[0], w.dz, w.dr)
    if ordered:  # z order: blocks read their nodes from LDS tiles
        s = s[np.argsort(s[:, 0], kind="stable")]
    got = run(w, states, s, precision)
    want = oracle.gather(grids(w), states, s)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    log(f"gather order {order} precision {precision} ordered {ordered}: max error {err:.2e} of the field scale")
    assert err < (1e-12 if precision == F.FP64 else 1e-5)


def test_gather_exact_for_linear_fields():
    w = workload([0, 1], 8, nz=90, nr=36)
    rng = np.random.default_rng(7)
    Fs = [rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)) for _ in range(2)]
    gs = grids(w)
    states = [staggered_state(g, Fm) for g, Fm in zip(gs, Fs)]
    nd = 4
    z = rng.uniform((nd + 3) * w.dz, (w.nz[0] - nd - 4) * w.dz, 2000)
    r = rng.uniform(0, (w.nr[0] - nd - 3) * w.dr, 2000)
    th = rng.uniform(-math.pi, math.pi, 2000)
    s = np.stack([z, r * np.cos(th), r * np.sin(th), np.ones(2000)], axis=1)
    got = run(w, states, s, F.FP64)
    for c in range(6):
        want = 0.0
        for m, Fm in ((0, Fs[0]), (1, Fs[1])):
            pS = 1 if m % 2 == 0 else -1
            pA = 1 if abs(m - 1) % 2 == 0 else -1
            odd = (pA if POLAR[c] else pS) == -1
            want = want + np.real((r if odd else 1.0) * (Fm[c, 0] + Fm[c, 1] * z / 5) * np.exp(1j * m * th))
        assert np.max(np.abs(got[:, c] - want)) < 1e-11 * max(1.0, np.max(np.abs(want))), c


def test_gather_after_steps_and_argument_checks():
    import torch
    w = workload([0, 1], 8)
    rng = np.random.default_rng(3)
    psi0 = [rng.uniform(-1, 1, (6, w.nr[0], w.nz[0])) + 1j * rng.uniform(-1, 1, (6, w.nr[0], w.nz[0]))
            for _ in range(w.n)]
    s = samples(rng, 2000, w.nz[0], w.nr[0], w.dz, w.dr)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        psi = [dev(x, torch.complex128) for x in psi0]
        plan = F.Plan(w.problems(), precision=F.FP64, flags=F.PLAN_USE_GRAPH)
        plan.step(psi, None, n_steps=2)
        out = plan.gather(psi, dev(s, torch.float64))
        torch.cuda.synchronize()
        stepped = [x.cpu().numpy() for x in psi]
        got = out.cpu().numpy()
        with pytest.raises(F.FdetdError):
            F.fdetd_gather(plan._h, [x.data_ptr() for x in psi], 0, 10, 0)  # NULL samples
        # no samples: nothing to do, plain or supersampled
        empty = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
        for ss in (0, 1, 2, 3):
            assert plan.gather(psi, empty, supersample=ss).shape == (0, 6)
        torch.cuda.synchronize()
        plan.close()
    want = oracle.gather(grids(w), stepped, s)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    # problems that are not modes of one grid
    w2 = I.Workload("two", 0, [100, 120], [30, 30], [0, 1], [8, 8], 8, w.dz, w.dr, w.dt, 1)
    plan = F.Plan(w2.problems(), precision=F.FP64, flags=F.PLAN_SKIP_STABILITY)
    with pytest.raises(F.FdetdError):
        plan.gather([torch.zeros((6, 30, 100), dtype=torch.complex128, device="cuda"),
                     torch.zeros((6, 30, 120), dtype=torch.complex128, device="cuda")],
                    torch.zeros((4, 4), dtype=torch.float64, device="cuda"))
    plan.close()


def bunch(rng, n, nz, dz, dr):
    """A compact bunch in z order (the LDS-tile path): z over 12 cells mid-grid, rho within 8 rows, a fifth
    of the samples next to the axis."""
    z = np.sort(rng.uniform(0.4 * nz * dz, (0.4 * nz + 12) * dz, n))
    r = np.sqrt(rng.uniform(0, 64, n)) * dr
    r[rng.random(n) < 0.2] = rng.uniform(0, 1.5 * dr)
    th = rng.uniform(-math.pi, math.pi, n)
    return np.stack([z, r * np.cos(th), r * np.sin(th), np.ones(n)], axis=1)


@pytest.mark.parametrize("ordered", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("order", [8, 16])
def test_supersampled_gather_matches_oracle(precision, order, ordered):
    """One plan, the three doublings in turn and the plain gather after them (the doubled-grid planes are
    reused across calls).  Unordered samples spread over the grid read the planes; a z-ordered compact
    bunch goes through the LDS tiles."""
    import torch
    w = workload([0, 1, 2], order)
    rng = np.random.default_rng(40 + order + precision)
    states = [rng.uniform(-1, 1, (6, w.nr[0], w.nz[0])) + 1j * rng.uniform(-1, 1, (6, w.nr[0], w.nz[0]))
              for _ in range(w.n)]
    s = bunch(rng, 6000, w.nz[0], w.dz, w.dr) if ordered else samples(rng, 3000, w.nz[0], w.nr[0], w.dz, w.dr)
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY)
    psi = [dev(x, cd) for x in states]
    sd = dev(s, torch.float64)
    for ss in (1, 2, 3, 0):
        got = plan.gather(psi, sd, supersample=ss).cpu().numpy()
        want = oracle.gather_fine(grids(w), states, s, ss)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        log(f"supersampled gather {ss} order {order} precision {precision} ordered {ordered}: max error {err:.2e} "
            f"of the field scale")
        assert err < (1e-12 if precision == F.FP64 else 1e-5), ss
    with pytest.raises(F.FdetdError):
        plan.gather(psi, sd, supersample=4)
    plan.close()


@pytest.mark.parametrize("ss", [1, 2, 3])
def test_supersampled_gather_exact_for_linear_fields(ss):
    w = workload([0, 1], 8, nz=90, nr=36)
    rng = np.random.default_rng(70 + ss)
    Fs = [rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)) for _ in range(2)]
    gs = grids(w)
    states = [staggered_state(g, Fm) for g, Fm in zip(gs, Fs)]
    nd = 4
    z = rng.uniform((nd + 3) * w.dz, (w.nz[0] - nd - 4) * w.dz, 2000)
    r = rng.uniform(0, (w.nr[0] - nd - 3) * w.dr, 2000)
    r[:300] = rng.uniform(0, 1.5 * w.dr, 300)  # nodes on and below the axis
    th = rng.uniform(-math.pi, math.pi, 2000)
    s = np.stack([z, r * np.cos(th), r * np.sin(th), np.ones(2000)], axis=1)
    got = run(w, states, s, F.FP64, supersample=ss)
    for c in range(6):
        want = 0.0
        for m, Fm in ((0, Fs[0]), (1, Fs[1])):
            pS = 1 if m % 2 == 0 else -1
            pA = 1 if abs(m - 1) % 2 == 0 else -1
            odd = (pA if POLAR[c] else pS) == -1
            want = want + np.real((r if odd else 1.0) * (Fm[c, 0] + Fm[c, 1] * z / 5) * np.exp(1j * m * th))
        assert np.max(np.abs(got[:, c] - want)) < 1e-11 * max(1.0, np.max(np.abs(want))), (ss, c)


@pytest.mark.parametrize("precision", [0, 1])
def test_gather_minimal_grids(precision):
    """The smallest grids a plan accepts (nz = 2 N_D + 1, nr = N_D + 1): every stencil and the axis rule
    reach the grid edges; plain and supersampled gathers against the oracle."""
    import torch
    for order in (2, 8, 32):
        nd = order // 2
        w = workload([0, 1, 2], order, nz=2 * nd + 1, nr=nd + 1)
        rng = np.random.default_rng(order + 10 * precision)
        states = [rng.uniform(-1, 1, (6, w.nr[0], w.nz[0])) + 1j * rng.uniform(-1, 1, (6, w.nr[0], w.nz[0]))
                  for _ in range(w.n)]
        s = samples(rng, 1500, w.nz[0], w.nr[0], w.dz, w.dr)
        cd = torch.complex128 if precision == F.FP64 else torch.complex64
        plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_SKIP_STABILITY | F.PLAN_NO_AUTOTUNE)
        psi = [dev(x, cd) for x in states]
        sd = dev(s, torch.float64)
        for ss in (0, 1, 2, 3):
            got = plan.gather(psi, sd, supersample=ss).cpu().numpy()
            want = oracle.gather_fine(grids(w), states, s, ss)
            err = np.max(np.abs(got - want)) / np.max(np.abs(want))
            assert err < (1e-12 if precision == F.FP64 else 1e-5), (order, ss, err)
        plan.close()
