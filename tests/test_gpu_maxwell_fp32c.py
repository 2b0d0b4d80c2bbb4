"""FP32-compensated path (float fields, float compensation words, FP64 arithmetic on the near-axis
segments) against the FP64 oracle, and the state export/import that makes it resumable.

Tolerance: helpers.tol_fp32c(steps, N) = 2 u (1 + 2 sqrt(N steps)), u = 2^-24 (4 sqrt for the envelope): each
Horner stage's increment carries a rounding of a few u of the terms it sums, the N stages of K steps add
like a random walk, and the compensated accumulation keeps the stored state's rounding (otherwise u/2 per
step) out of the sum.  Measured 7e-8 .. 5e-7 on these runs, a tenth to a quarter of the bound.
"""
import numpy as np
import pytest

from helpers import dev, gpu_envelope, gpu_maxwell, log, oracle_envelope, oracle_maxwell, rel_l2, tol_fp32c

import paper_2605_12132_amd as F
import paper_2605_12132_amd.inputs as I

pytestmark = pytest.mark.gpu



def small(m, order, N, nz=150, nr=37, steps=1):
    dz = I.LAMBDA0 / 20
    return I.Workload(f"small32_m{m}_o{order}", 0, [nz], [nr], [m], [order], N, dz, 2 * dz, 0.5 * dz, steps)


@pytest.mark.parametrize("m,order,N", [(0, 8, 8), (1, 16, 8), (2, 32, 4), (1, 2, 1)])
def test_fp32c_matches_oracle(m, order, N):
    w = small(m, order, N, steps=3)
    rng = np.random.default_rng(31 + m + order)
    psi0 = [rng.uniform(-1, 1, (6, 37, 150)) + 1j * rng.uniform(-1, 1, (6, 37, 150))]
    J = [0.1 * (rng.uniform(-1, 1, (3, 3, 37, 150)) + 1j * rng.uniform(-1, 1, (3, 3, 37, 150)))]
    log(f"fp32c m={m} order={order} N={N}")
    got, _ = gpu_maxwell(w, psi0, J, 3, precision=F.FP32C, flags=1)
    want = oracle_maxwell(w, psi0, J, 3)
    err = rel_l2(got[0], want[0])
    log(f"  rel L2 {err:.3e} (bound {tol_fp32c(3, N):.2e})")
    assert err < tol_fp32c(3, N)


def test_fp32c_without_source_and_graph():
    w = I.vacuum_pulse().shrink(steps=20)
    psi0 = [I.initial_fields(w, 0)]
    eager, _ = gpu_maxwell(w, psi0, None, 20, precision=F.FP32C)
    graph, _ = gpu_maxwell(w, psi0, None, 20, precision=F.FP32C, flags=2)
    assert np.array_equal(eager[0], graph[0])
    want = oracle_maxwell(w, psi0, None, 20)
    err = rel_l2(eager[0], want[0])
    log(f"fp32c vacuum pulse, 20 steps: rel L2 {err:.3e} (bound {tol_fp32c(20, w.taylor_order):.2e})")
    assert err < tol_fp32c(20, w.taylor_order)


@pytest.mark.parametrize("order,m", [(8, 0), (24, 1)])
def test_fp32c_envelope_matches_oracle(order, m):
    """Order 8: near-axis tiles with a whole complex value per lane; order 24: read in lane pairs."""
    dz = I.LAMBDA0 / 5
    w = I.Workload("env32", 1, [203], [41], [m], [order], 4, dz, 0.2 * I.UM, 0.5 * dz, 10, seed=8,
                   extra=dict(a0=2.0, w0=4 * I.UM, ctau=3 * I.UM, zc=10 * I.UM, chi0=1e-3, mod=0.05))
    a0, at0 = I.envelope_initial(w)
    chi = I.envelope_chi(w)
    ga, gt, _ = gpu_envelope(w, [a0], [at0], [chi], 10, precision=F.FP32C, flags=1)
    oa, ot = oracle_envelope(w, [a0], [at0], [chi], 10)
    err = rel_l2(np.concatenate([ga[0].ravel(), gt[0].ravel()]), np.concatenate([oa[0].ravel(), ot[0].ravel()]))
    log(f"fp32c envelope order {order}, 10 steps: rel L2 {err:.3e} (bound {tol_fp32c(10, 4, envelope=True):.2e})")
    assert err < tol_fp32c(10, 4, envelope=True)


def test_export_import_resume_is_bitwise():
    """2K steps in one plan == K steps, export the compensation words, a new plan imports them, K steps."""
    import torch
    w = small(1, 8, 8, steps=4)
    rng = np.random.default_rng(77)
    psi0 = rng.uniform(-1, 1, (6, 37, 150)) + 1j * rng.uniform(-1, 1, (6, 37, 150))
    J = 0.1 * (rng.uniform(-1, 1, (4, 3, 37, 150)) + 1j * rng.uniform(-1, 1, (4, 3, 37, 150)))
    jd = dev(J, torch.complex64)
    a = dev(psi0, torch.complex64)
    pa = F.Plan(w.problems(), precision=F.FP32C, flags=1)
    pa.step([a], [jd], n_steps=4)
    b = dev(psi0, torch.complex64)
    pb = F.Plan(w.problems(), precision=F.FP32C, flags=1)
    pb.step([b], [jd[:2]], n_steps=2)
    blob = pb.export_state()
    assert len(blob) == 6 * 37 * 150 * 8
    saved = b.clone()
    pb.close()
    c = saved.clone()
    pc = F.Plan(w.problems(), precision=F.FP32C, flags=1)
    pc.import_state(blob)                   # the next call adopts the words for its pointers
    pc.step([c], [jd[2:]], n_steps=2)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    # FP64 plans carry no state
    p64 = F.Plan(w.problems(), precision=F.FP64, flags=1)
    assert p64.export_state() == b""
    for p in (pa, pc, p64):
        p.close()


@pytest.mark.parametrize("order,nr,nz", [(32, 20, 70), (16, 20, 33), (4, 8, 9)])
def test_fp32c_grid_all_near_axis(order, nr, nz):
    """Grids with fewer than 2 N_D rows: every row is a near-axis row (FP64 arithmetic), the launch has
    near-axis tiles only; minimal z extents included (N_z = 2 N_D + 1)."""
    w = small(1, order, 8, nz=nz, nr=nr, steps=2)
    rng = np.random.default_rng(order + nr)
    psi0 = [rng.uniform(-1, 1, (6, nr, nz)) + 1j * rng.uniform(-1, 1, (6, nr, nz))]
    J = [0.1 * (rng.uniform(-1, 1, (2, 3, nr, nz)) + 1j * rng.uniform(-1, 1, (2, 3, nr, nz)))]
    got, info = gpu_maxwell(w, psi0, J, 2, precision=F.FP32C, flags=1)
    want = oracle_maxwell(w, psi0, J, 2)
    err = rel_l2(got[0], want[0])
    log(f"fp32c all near-axis order {order} {nz}x{nr}: rel L2 {err:.2e}")
    assert err < tol_fp32c(2, 8)


def test_fp32c_element_alignment():
    """FP32C buffers need only their element's alignment (8 bytes): with an odd cell count the current of
    step 1 starts 8 bytes past a 16-byte boundary and is accepted; a pointer 4 bytes off is rejected on the
    host before anything is enqueued."""
    import torch
    from paper_2605_12132_amd import binding as B
    w = small(1, 8, 4, nz=151, nr=37, steps=2)
    assert (3 * 37 * 151 * 8) % 16 == 8
    rng = np.random.default_rng(5)
    psi0 = rng.uniform(-1, 1, (6, 37, 151)) + 1j * rng.uniform(-1, 1, (6, 37, 151))
    J = 0.1 * (rng.uniform(-1, 1, (3, 3, 37, 151)) + 1j * rng.uniform(-1, 1, (3, 3, 37, 151)))
    jd = dev(J, torch.complex64)
    psi = dev(psi0, torch.complex64)
    plan = F.Plan(w.problems(), precision=F.FP32C, flags=1)
    assert jd[1:].data_ptr() % 16 == 8
    plan.step([psi], [jd[1:]], n_steps=2)
    torch.cuda.synchronize()
    want = oracle_maxwell(w, [psi0], [J[1:]], 2)
    assert rel_l2(psi.cpu().numpy().astype(np.complex128), want[0]) < tol_fp32c(2, 4)
    with pytest.raises(F.FdetdError) as e:
        B.fdetd_step(plan._h, [psi.data_ptr() + 4], None, 0, 1)
    assert e.value.code == -1 and "aligned" in str(e.value)
    plan.close()
