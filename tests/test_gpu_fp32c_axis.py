"""FP32C error split by rows, against the FP64 oracle: the near-axis rows k < 2 N_D (their stencils reach
the mirrored rows below the axis and the largest 1/rho factors: rho^-1 D(rho F) divides differences of
rho F, up to (2 N_D + 1) dr across, by rho_k = dr/2 on the first row) and the rows further out.  With
the default FP64 arithmetic on those rows, and with FDETD_AXIS_ROWS=0 (float arithmetic everywhere), on
random fields with a random current (the worst case for cancellation) over 5 steps.

The FP64 band must keep the near-axis rows as accurate as the rest (within 2x of the outer rows' error);
the float-only variant shows what the band buys (logged, and required to be no better on those rows)."""
import os

import numpy as np
import pytest

from helpers import gpu_maxwell, log, oracle_maxwell, rel_l2

import paper_2605_12132_amd as F
import paper_2605_12132_amd.inputs as I

pytestmark = pytest.mark.gpu


class axis_rows_env:
    def __init__(self, n):
        self.n, self.old = n, None

    def __enter__(self):
        self.old = os.environ.get("FDETD_AXIS_ROWS")
        os.environ["FDETD_AXIS_ROWS"] = str(self.n)

    def __exit__(self, *a):
        if self.old is None:
            del os.environ["FDETD_AXIS_ROWS"]
        else:
            os.environ["FDETD_AXIS_ROWS"] = self.old
        return False


def split_errors(got, want, rows):
    return rel_l2(got[:, :rows], want[:, :rows]), rel_l2(got[:, rows:], want[:, rows:])


@pytest.mark.parametrize("m,order", [(0, 8), (1, 16), (2, 32), (1, 32)])
def test_near_axis_rows_error(m, order):
    dz = I.LAMBDA0 / 20
    nz, nr, steps = 160, 96, 5
    w = I.Workload(f"axis_m{m}_o{order}", 0, [nz], [nr], [m], [order], 8, dz, 2 * dz, 0.5 * dz, steps)
    rng = np.random.default_rng(1000 + 10 * m + order)
    psi0 = [rng.uniform(-1, 1, (6, nr, nz)) + 1j * rng.uniform(-1, 1, (6, nr, nz))]
    J = [0.1 * (rng.uniform(-1, 1, (steps, 3, nr, nz)) + 1j * rng.uniform(-1, 1, (steps, 3, nr, nz)))]
    want = oracle_maxwell(w, psi0, J, steps)[0]
    rows = order  # 2 N_D
    band, _ = gpu_maxwell(w, psi0, J, steps, precision=F.FP32C, flags=F.PLAN_SKIP_STABILITY)
    with axis_rows_env(0):
        flt, _ = gpu_maxwell(w, psi0, J, steps, precision=F.FP32C, flags=F.PLAN_SKIP_STABILITY)
    ea, em = split_errors(band[0], want, rows)
    fa, fm = split_errors(flt[0], want, rows)
    log(f"m={m} order {order}: FP64 band: near-axis rows {ea:.2e}, outer rows {em:.2e}; "
        f"float only: near-axis {fa:.2e}, outer {fm:.2e} (x{fa / ea:.1f} near the axis)")
    assert ea < 2 * em
    assert fa >= 0.9 * ea
