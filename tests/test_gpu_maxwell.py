"""GPU parity of the Maxwell field update (HIP library through the C-ABI) against the CPU FP64 oracle.

Both sides receive the same seeded inputs from paper_2605_12132_amd.inputs; the oracle evaluates the
paper's forward Taylor sums (2N applications of H per step with a source), the GPU a Horner recurrence
(N applications) -- the same polynomial, so the FP64 results agree to rounding.  Tolerance: relative L2
<= 1e-12 over all six components (rounding of both sides grows ~sqrt(steps) * N * eps * ||H|| dt).
Grids span several 64 x 4 workgroup tiles with ragged tails in both directions.
"""
import numpy as np
import pytest

from helpers import gpu_maxwell, log, oracle_maxwell, rel_l2

import paper_2605_12132_amd.inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def small(m, order, N, nz=150, nr=37, steps=1, dt_factor=0.5, seed=0):
    dz = I.LAMBDA0 / 20
    return I.Workload(f"small_m{m}_o{order}", 0, [nz], [nr], [m], [order], N, dz, 2 * dz, dt_factor * dz, steps,
                      seed=seed)


def random_state(w, p, rng):
    x = rng.uniform(-1, 1, (6, w.nr[p], w.nz[p])) + 1j * rng.uniform(-1, 1, (6, w.nr[p], w.nz[p]))
    return x


def random_current(w, p, steps, rng):
    return 0.1 * (rng.uniform(-1, 1, (steps, 3, w.nr[p], w.nz[p])) + 1j * rng.uniform(-1, 1, (steps, 3, w.nr[p], w.nz[p])))


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [2, 8, 16, 32])
def test_single_stage_random_state(m, order):
    # N = 1: psi' = psi + dt (H psi - Jbar): one application of the operator, every row and column
    w = small(m, order, 1)
    rng = np.random.default_rng(100 + m * 40 + order)
    psi0 = [random_state(w, 0, rng)]
    J = [random_current(w, 0, 1, rng)]
    log(f"single stage m={m} order={order} {w.nz[0]}x{w.nr[0]}")
    got, _ = gpu_maxwell(w, psi0, J, 1, flags=1)
    want = oracle_maxwell(w, psi0, J, 1)
    assert rel_l2(got[0], want[0]) < 1e-13


@pytest.mark.parametrize("m,order,N", [(1, 8, 4), (0, 16, 8)])
def test_steps_without_source(m, order, N):
    w = small(m, order, N, steps=2)
    rng = np.random.default_rng(3 + m + order)
    psi0 = [random_state(w, 0, rng)]
    log(f"2 steps without current m={m} order={order} N={N}")
    got, _ = gpu_maxwell(w, psi0, None, 2, flags=1)
    want = oracle_maxwell(w, psi0, None, 2)
    assert rel_l2(got[0], want[0]) < TOL64


@pytest.mark.parametrize("m,order,N", [(0, 4, 8), (1, 16, 8), (2, 32, 8), (3, 8, 12), (1, 6, 4), (5, 10, 8)])
def test_steps_with_source(m, order, N):
    w = small(m, order, N, steps=3)
    rng = np.random.default_rng(7 + m + order)
    psi0 = [random_state(w, 0, rng)]
    J = [random_current(w, 0, 3, rng)]
    log(f"3 steps m={m} order={order} N={N}")
    got, _ = gpu_maxwell(w, psi0, J, 3, flags=1)
    want = oracle_maxwell(w, psi0, J, 3)
    assert rel_l2(got[0], want[0]) < TOL64


def test_vacuum_pulse_full_run():
    """m = 1 pulse, 256 x 64, order 8, Taylor 12, dt = dz, 100 steps (the plan's stability check on)."""
    w = I.vacuum_pulse()
    psi0 = [I.initial_fields(w, 0)]
    log("vacuum pulse 100 steps")
    got, info = gpu_maxwell(w, psi0, None, w.steps)
    assert 0 < info["dt_rho_max"] < 3.38
    want = oracle_maxwell(w, psi0, None, w.steps)
    err = rel_l2(got[0], want[0])
    log(f"vacuum pulse rel L2 {err:.3e}")
    assert err < TOL64


def test_current_driven_full_size_graph():
    """Both modes at full size (2048 x 256, order 16) for 3 steps with the bunch current, in the
    configuration the benchmark times (hipGraph replay)."""
    w = I.current_driven()
    steps = 3
    psi0 = [np.zeros((6, w.nr[p], w.nz[p]), np.complex128) + I.noise((6, w.nr[p], w.nz[p]), 1e-3,
                                                                   np.random.default_rng(p), real_only=w.m[p] == 0)
            for p in range(w.n)]
    J = [I.currents(w, p, steps) for p in range(w.n)]
    log("current-driven full size, 3 steps, graph")
    got, _ = gpu_maxwell(w, psi0, J, steps, flags=2)
    want = oracle_maxwell(w, psi0, J, steps)
    for p in range(w.n):
        err = rel_l2(got[p], want[p])
        log(f"  mode {w.m[p]} rel L2 {err:.3e}")
        assert err < TOL64


def test_batched_uneven_first_problems():
    """Six problems of the uneven batch (different grids, modes and orders) in one plan, 2 steps."""
    full = I.batched_uneven()
    idx = list(range(6))
    w = I.Workload(full.name, 0, [full.nz[p] for p in idx], [full.nr[p] for p in idx], [full.m[p] for p in idx],
                   [full.fd_order[p] for p in idx], full.taylor_order, full.dz, full.dr, full.dt, 2, seed=full.seed,
                   extra=full.extra)
    psi0 = [I.initial_fields(w, p) for p in range(w.n)]
    J = [I.currents(w, p, 2) for p in range(w.n)]
    log("batched uneven, 6 problems, 2 steps")
    got, _ = gpu_maxwell(w, psi0, J, 2)
    want = oracle_maxwell(w, psi0, J, 2)
    for p in range(w.n):
        err = rel_l2(got[p], want[p])
        log(f"  problem {p} {w.nz[p]}x{w.nr[p]} m={w.m[p]} order={w.fd_order[p]} rel L2 {err:.3e}")
        assert err < TOL64


def test_minimal_grids_and_low_orders():
    for order in (2, 4, 32):
        nd = order // 2
        w = small(1, order, 4, nz=2 * nd + 1, nr=nd + 1, steps=2)
        rng = np.random.default_rng(order)
        psi0 = [random_state(w, 0, rng)]
        J = [random_current(w, 0, 2, rng)]
        got, _ = gpu_maxwell(w, psi0, J, 2, flags=1)
        want = oracle_maxwell(w, psi0, J, 2)
        assert rel_l2(got[0], want[0]) < TOL64, order


def test_batched_equals_single_bitwise_and_graph_equals_eager():
    ws = [small(0, 8, 8, nz=300, nr=70, steps=2, seed=1), small(2, 12, 8, nz=130, nr=19, steps=2, seed=2),
          small(1, 32, 8, nz=517, nr=33, steps=2, seed=3)]
    rng = np.random.default_rng(55)
    psi0 = [random_state(w, 0, rng) for w in ws]
    J = [random_current(w, 0, 2, rng) for w in ws]
    batch = I.Workload("mix", 0, [w.nz[0] for w in ws], [w.nr[0] for w in ws], [w.m[0] for w in ws],
                       [w.fd_order[0] for w in ws], 8, ws[0].dz, ws[0].dr, ws[0].dt, 2)
    got_b, _ = gpu_maxwell(batch, psi0, J, 2, flags=1)
    for p, w in enumerate(ws):
        got_s, _ = gpu_maxwell(w, [psi0[p]], [J[p]], 2, flags=1)
        assert np.array_equal(got_b[p], got_s[0])
    eager, _ = gpu_maxwell(ws[2], [psi0[2]], [J[2]], 2, flags=1)
    graph, _ = gpu_maxwell(ws[2], [psi0[2]], [J[2]], 2, flags=3)
    assert np.array_equal(eager[0], graph[0])
    # two calls of one step each == one call of two steps (per-step current offsets)
    split, _ = gpu_maxwell(ws[2], [psi0[2]], [J[2]], 2, flags=1, calls=2)
    assert np.array_equal(eager[0], split[0])


def test_axis_slots_ignored_and_zero_steps():
    w = small(0, 8, 8, steps=1)
    rng = np.random.default_rng(9)
    psi0 = random_state(w, 0, rng)
    J = [random_current(w, 0, 1, rng)]
    a, _ = gpu_maxwell(w, [psi0], J, 1, flags=1)
    psi1 = psi0.copy()
    psi1[[0, 4, 5], 0, :] = 1e6
    b, _ = gpu_maxwell(w, [psi1], J, 1, flags=1)
    assert np.array_equal(a[0], b[0])
    c, _ = gpu_maxwell(w, [psi0], J, 0, flags=1)
    assert np.array_equal(c[0], psi0)


def test_single_hip_runtime_in_process():
    import torch  # noqa: F401
    import paper_2605_12132_amd  # noqa: F401
    maps = open("/proc/self/maps").read()
    hip = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hip) == 1, hip


@pytest.mark.parametrize("precision", [0, 1])
def test_tiling_and_autotune_do_not_change_results(precision, monkeypatch):
    """Every output is formed by the same operations whatever the marching segment length, so plans with
    forced segment lengths (main and, in FP32C, near-axis tiles), store policies of the stage outputs or
    tile orders, the default and the autotuned one give bitwise equal fields (FP64 and FP32C, eager and
    graph)."""
    import paper_2605_12132_amd as F
    w = small(1, 16, 8, nz=300, nr=90, steps=2, seed=4)
    rng = np.random.default_rng(71)
    psi0 = [random_state(w, 0, rng)]
    J = [random_current(w, 0, 2, rng)]
    runs = {}
    for seg in ("1", "5", "64"):
        monkeypatch.setenv("FDETD_SEG_ROWS", seg)
        runs[seg], info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=1)
        assert info["seg_rows"] == int(seg) and info["autotune_ms"] == 0.0
    monkeypatch.delenv("FDETD_SEG_ROWS")
    runs["default"], _ = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=1 | F.PLAN_NO_AUTOTUNE)
    runs["tuned"], info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=1)
    runs["graph"], _ = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=3)
    log(f"autotuned: {info['seg_rows']} rows per segment (near-axis {info['seg_rows_axis']}), {info['autotune_ms']:.1f} ms")
    assert info["seg_rows"] in (8, 16, 32, 64, 128, 256) and info["autotune_ms"] > 0
    assert info["seg_rows_axis"] == (0 if precision == 0 else 16)  # min(16, 2 N_D) for order 16
    if precision == 1:  # the near-axis segment length (FP32C) does not change results either
        for sa in ("1", "5", "32"):
            monkeypatch.setenv("FDETD_SEG_AXIS", sa)
            runs["axis" + sa], info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=1 | F.PLAN_NO_AUTOTUNE)
            assert info["seg_rows_axis"] == min(int(sa), 16)
        monkeypatch.delenv("FDETD_SEG_AXIS")
    for pol in ("0", "1"):  # the store policy of the stage outputs changes no value either
        monkeypatch.setenv("FDETD_STORE_POLICY", pol)
        runs["store" + pol], info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=1)
        assert info["store_policy"] == int(pol)
    monkeypatch.delenv("FDETD_STORE_POLICY")
    for order in ("0", "1"):  # nor the numbering of the tiles
        monkeypatch.setenv("FDETD_TILE_ORDER", order)
        runs["order" + order], info = gpu_maxwell(w, psi0, J, 2, precision=precision, flags=3)
        assert info["tile_order"] == int(order)
    monkeypatch.delenv("FDETD_TILE_ORDER")
    for k, v in runs.items():
        assert np.array_equal(v[0], runs["1"][0]), k
    if precision == 0:
        assert rel_l2(runs["1"][0], oracle_maxwell(w, psi0, J, 2)[0]) < TOL64


def test_graph_recaptures_when_pointers_change():
    """A graph plan replays its captured graph only for the exact previous call (same pointers, step count,
    current stride); other calls capture anew.  Alternating two state buffers and step counts gives the
    eager results each time."""
    import torch
    import paper_2605_12132_amd as F
    from helpers import dev
    w = small(1, 8, 8, nz=160, nr=40, steps=3, seed=6)
    rng = np.random.default_rng(12)
    psi0 = random_state(w, 0, rng)
    J = random_current(w, 0, 3, rng)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        jd = dev(J, torch.complex128)
        a, b = dev(psi0, torch.complex128), dev(psi0, torch.complex128)
        g = F.Plan(w.problems(), precision=F.FP64, flags=F.PLAN_USE_GRAPH | 1)
        e = F.Plan(w.problems(), precision=F.FP64, flags=1)
        ea, eb = dev(psi0, torch.complex128), dev(psi0, torch.complex128)
        for x, ex, n in ((a, ea, 1), (b, eb, 1), (a, ea, 1), (a, ea, 2), (b, eb, 2), (b, eb, 2)):
            g.step([x], [jd], n_steps=n)
            e.step([ex], [jd], n_steps=n)
        torch.cuda.synchronize()
        assert torch.equal(a, ea) and torch.equal(b, eb)
        g.close()
        e.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_concurrent_batches_equal_one_stream(precision):
    """A plan with five launch batches (five stencil widths) runs them on four streams.  Batches hold
    disjoint problems, so the fields equal, bitwise, those of the same plan on one stream.  A graph plan
    (one branch per stream) replayed over several calls, with eager work of another plan and
    synchronisation between the replays, matches the eager plan after every call."""
    import torch
    import paper_2605_12132_amd as F
    from helpers import dev
    ws = [small(0, 8, 8, nz=300, nr=70, steps=3, seed=11), small(2, 12, 8, nz=130, nr=19, steps=3, seed=12),
          small(1, 32, 8, nz=517, nr=33, steps=3, seed=13), small(1, 4, 8, nz=257, nr=45, steps=3, seed=14),
          small(0, 16, 8, nz=180, nr=64, steps=3, seed=15), small(3, 8, 8, nz=96, nr=30, steps=3, seed=16)]
    rng = np.random.default_rng(77)
    psi0 = [random_state(w, 0, rng) for w in ws]
    J = [random_current(w, 0, 3, rng) for w in ws]
    batch = I.Workload("mix5", 0, [w.nz[0] for w in ws], [w.nr[0] for w in ws], [w.m[0] for w in ws],
                       [w.fd_order[0] for w in ws], 8, ws[0].dz, ws[0].dr, ws[0].dt, 3)
    pw = F.PLAN_PER_WIDTH
    lanes, info = gpu_maxwell(batch, psi0, J, 3, precision=precision, flags=1 | pw)
    one, info1 = gpu_maxwell(batch, psi0, J, 3, precision=precision, flags=1 | pw | F.PLAN_ONE_STREAM)
    log(f"five batches: {info['streams']} streams, one-stream plan {info1['streams']}")
    assert info["streams"] == 4 and info1["streams"] == 1
    for p in range(batch.n):
        assert np.array_equal(lanes[p], one[p]), p
    if precision == 0:
        want = oracle_maxwell(batch, psi0, J, 3)
        for p in range(batch.n):
            assert rel_l2(lanes[p], want[p]) < TOL64, p
    cd = torch.complex128 if precision == 0 else torch.complex64
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        jd = [dev(j, cd) for j in J]
        g_psi = [dev(x, cd) for x in psi0]
        e_psi = [dev(x, cd) for x in psi0]
        g = F.Plan(batch.problems(), precision=precision, flags=F.PLAN_USE_GRAPH | 1 | pw)
        e = F.Plan(batch.problems(), precision=precision, flags=1 | pw)
        assert g.query()["streams"] == 4
        for call in range(4):  # the same pointers each call: one capture, then replays
            g.step(g_psi, [j[0] for j in jd], n_steps=1)
            torch.cuda.synchronize()
            e.step(e_psi, [j[0] for j in jd], n_steps=1)
            torch.cuda.synchronize()
            for p in range(batch.n):
                assert torch.equal(g_psi[p], e_psi[p]), (call, p)
        g.close()
        e.close()
