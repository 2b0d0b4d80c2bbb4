"""Mixed-width launch batches (the FP64 default, FDETD_PLAN_MIXED_WIDTHS for FP32C): one launch batch for
problems of every stencil width (each tile runs the code of its problem's width), against the per-width
batches (FDETD_PLAN_PER_WIDTH) on up to four streams.  The same code runs on the
same data in the same order per output value, so the states agree bit for bit, in FP64 and FP32C, with
resident currents and with the current made in the captured time loop; the launch counts drop to N + 1
per step with a current (the staged J_rho and N stages; FP32C: 2 N + 1, the near-axis tiles in a launch of
their own)."""
import numpy as np
import pytest

from helpers import dev, gpu_maxwell, log

import paper_2605_12132_amd as F
import paper_2605_12132_amd.inputs as I

pytestmark = pytest.mark.gpu


def subset(n=14):
    w = I.batched_uneven()
    keep = list(range(n))
    return I.Workload("mixed_subset", 0, [w.nz[p] // 2 for p in keep], [w.nr[p] // 2 for p in keep],
                      [w.m[p] for p in keep], [w.fd_order[p] for p in keep], w.taylor_order, w.dz, w.dr, w.dt, 3,
                      seed=w.seed, extra=w.extra)


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_widths_equal_per_width_batches(precision):
    w = subset()
    assert len(set(w.fd_order)) > 4
    steps = 3
    psi0 = [I.initial_fields(w, p) for p in range(w.n)]
    J = [I.currents(w, p, steps) for p in range(w.n)]
    per, info_p = gpu_maxwell(w, psi0, J, steps, precision=precision, flags=F.PLAN_USE_GRAPH | F.PLAN_PER_WIDTH)
    mix, info_m = gpu_maxwell(w, psi0, J, steps, precision=precision, flags=F.PLAN_USE_GRAPH | F.PLAN_MIXED_WIDTHS)
    dflt, info_d = gpu_maxwell(w, psi0, J, steps, precision=precision, flags=F.PLAN_USE_GRAPH)
    assert info_d["launches_per_step"] == (info_m if precision == F.FP64 else info_p)["launches_per_step"]
    log(f"precision {precision}: per-width {info_p['launches_per_step']} launches/step on {info_p['streams']} streams, "
        f"mixed {info_m['launches_per_step']} on {info_m['streams']}")
    N = w.taylor_order
    assert info_m["streams"] == 1
    assert info_m["launches_per_step"] == (N + 1 if precision == F.FP64 else 2 * N + 1)
    assert info_p["streams"] == 4
    for p in range(w.n):
        assert np.array_equal(per[p], mix[p]) and np.array_equal(per[p], dflt[p]), p


def test_mixed_widths_with_generated_current():
    import torch
    w = subset(10)
    e = w.extra
    jg = F.Jgen(F.JGEN_BUNCH, step0=2, seed=w.seed, nb=e["nb"], sigz=e["sigz"], sigr=e["sigr"], noise=e["noise"])
    outs = []
    for flags in (F.PLAN_USE_GRAPH | F.PLAN_PER_WIDTH, F.PLAN_USE_GRAPH | F.PLAN_MIXED_WIDTHS):
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            plan = F.Plan(w.problems(), precision=F.FP64, flags=flags)
            psi = [dev(I.initial_fields(w, p), torch.complex128) for p in range(w.n)]
            jw = [torch.zeros((3, w.nr[p], w.nz[p]), dtype=torch.complex128, device="cuda") for p in range(w.n)]
            plan.step_graph(psi, jg, jw, n_steps=4)
            torch.cuda.synchronize()
            plan.close()
        outs.append([x.cpu().numpy() for x in psi])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_widths_minimal_grids_against_the_oracle(precision):
    """One launch batch of minimal grids of every order 2..32 (N_z = 2 N_D + 1, N_rho = N_D + 1), modes 0..3:
    against the oracle (FP64 1e-12, FP32C the stated bound)."""
    from helpers import oracle_maxwell, rel_l2, tol_fp32c
    orders = list(range(2, 33, 2))
    dz = I.LAMBDA0 / 20
    w = I.Workload("mixed_min", 0, [o + 1 for o in orders], [o // 2 + 1 for o in orders], [k % 4 for k in range(16)],
                   orders, 8, dz, 2 * dz, 0.5 * dz, 2)
    rng = np.random.default_rng(3)
    psi0, J = [], []
    for p in range(w.n):
        shape = (6, w.nr[p], w.nz[p])
        x = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
        psi0.append(x.real + 0j if w.m[p] == 0 else x)
        j = 0.1 * (rng.uniform(-1, 1, (2, 3) + shape[1:]) + 1j * rng.uniform(-1, 1, (2, 3) + shape[1:]))
        J.append(j.real + 0j if w.m[p] == 0 else j)
    got, info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=F.PLAN_MIXED_WIDTHS | F.PLAN_SKIP_STABILITY)
    want = oracle_maxwell(w, psi0, J, 2)
    tol = 1e-12 if precision == F.FP64 else tol_fp32c(2, 8)
    worst = max(rel_l2(got[p], want[p]) for p in range(w.n))
    log(f"mixed-width minimal grids, precision {precision}: {info['launches_per_step']} launches per step, worst rel L2 {worst:.2e}")
    assert worst < tol
