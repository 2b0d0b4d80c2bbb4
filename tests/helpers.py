"""Shared helpers of the GPU tests: device transfers, running the library and the oracle on the same
seeded inputs, and the error measures the tolerances are stated in."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tol_fp32c(steps: int, taylor_order: int, envelope: bool = False) -> float:
    """Stated bound on the relative L2 error of the FP32-compensated path after `steps` steps of Taylor order
    N: every Horner stage forms its increment in float with a relative rounding of a few u = 2^-24 of the
    terms it sums (the coefficients carried in FP64), the compensated state keeps the stored value's
    rounding out of the sum, and the N K stage errors add like a random walk; the input and output rounding
    adds about u.  Bound: 2 u (1 + c sqrt(N K)), c = 2 for Maxwell.  The envelope takes c = 4: for a forward
    pulse its k0 terms 2 i k0 (D_z a + a~) nearly cancel to the envelope's small frequency shift, so each
    stage's rounding is relative to terms larger than the increment.  Measured: 0.1 to 0.4 of the bound
    (short runs, random fields), 0.3 (current-driven, 500 steps), 0.4 (envelope, 2000 steps)."""
    c = 4.0 if envelope else 2.0
    return 2.0 * 2.0 ** -24 * (1.0 + c * (steps * taylor_order) ** 0.5)


def rel_l2(got, want) -> float:
    got = np.asarray(got)
    want = np.asarray(want)
    den = np.linalg.norm(want.ravel())
    return float(np.linalg.norm((got - want).ravel()) / (den if den > 0 else 1.0))


def grid_of(w, p) -> oracle.Grid:
    return oracle.Grid(nz=w.nz[p], nr=w.nr[p], m=w.m[p], fd_order=w.fd_order[p], taylor_order=w.taylor_order,
                       dz=w.dz, dr=w.dr, dt=w.dt, k0=w.k0)


def dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()


def gpu_maxwell(w, psi0, J=None, steps=1, precision=0, flags=0, calls=1):
    """Run the library on all problems of workload w.  J: None or per-problem [steps, 3, nr, nz].
    `calls` splits the steps over that many fdetd_step calls (exercising per-call current offsets)."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    psi = [dev(x, cd) for x in psi0]
    jd = [dev(j, cd) for j in J] if J is not None else None
    stream = torch.cuda.Stream() if flags & F.PLAN_USE_GRAPH else None
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
    ctx = torch.cuda.stream(stream) if stream is not None else _null()
    with ctx:
        plan = F.Plan(w.problems(), precision=precision, flags=flags)
        per = steps // calls
        done = 0
        for c in range(calls):
            n = per if c < calls - 1 else steps - done
            plan.step(psi, [j[done:] for j in jd] if jd is not None else None, n_steps=n)
            done += n
        torch.cuda.synchronize()
        info = plan.query()
        plan.close()
    return [x.cpu().numpy().astype(np.complex128) for x in psi], info


def oracle_maxwell(w, psi0, J=None, steps=1):
    return [oracle.step(grid_of(w, p), psi0[p], None if J is None else J[p], steps) for p in range(w.n)]


class _null:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def gpu_envelope(w, a0, at0, chi, steps=1, precision=0, flags=0, absorbers=(), calls=1):
    """absorbers: (problem, lz, lr, sigma_max, power) layers set on the plan before stepping; `calls` splits
    the steps over that many envelope_step calls."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    rd = torch.float64 if precision == F.FP64 else torch.float32
    a = [dev(x, cd) for x in a0]
    at = [dev(x, cd) for x in at0]
    ch = [dev(x, rd) for x in chi]
    stream = torch.cuda.Stream() if flags & F.PLAN_USE_GRAPH else None
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
    ctx = torch.cuda.stream(stream) if stream is not None else _null()
    with ctx:
        plan = F.Plan(w.problems(), precision=precision, flags=flags)
        for p, lz, lr, smax, power in absorbers:
            plan.absorber(lz, lr, smax, power, problem=p)
        per = steps // calls
        for c in range(calls):
            plan.envelope_step(a, at, ch, n_steps=per if c < calls - 1 else steps - per * (calls - 1))
        torch.cuda.synchronize()
        info = plan.query()
        plan.close()
    return ([x.cpu().numpy().astype(np.complex128) for x in a], [x.cpu().numpy().astype(np.complex128) for x in at],
            info)


def oracle_envelope(w, a0, at0, chi, steps=1, absorbers=()):
    """absorbers as for gpu_envelope: those problems take the oracle's absorbing-layer step."""
    lay = {p: (lz, lr, smax, power) for p, lz, lr, smax, power in absorbers}
    out = []
    for p in range(w.n):
        g = grid_of(w, p)
        if p in lay:
            sigma = oracle.absorber_profile(g, *lay[p])
            out.append(oracle.envelope_step_absorbing(g, a0[p], at0[p], chi[p], sigma, steps))
        else:
            out.append(oracle.envelope_step(g, a0[p], at0[p], chi[p], steps))
    return [o[0] for o in out], [o[1] for o in out]


def dependence_radius(w, p, steps) -> int:
    """Cells (in z and rho) over which `steps` steps can carry information: each application of H reaches
    N_D cells, a step applies H up to N times to a vector that already holds the staged current (half-shift
    of N_D rows), plus a margin."""
    return steps * (w.taylor_order + 1) * (w.fd_order[p] // 2) + 2


def oracle_window(w, p, psi0, J, steps, zc, half, kmax):
    """The oracle on a crop of problem p -- rows [0, kr) and columns [z0, z1) -- that extends the sampled
    region (rows [0, kmax), columns [zc - half, zc + half)) by the dependence radius wherever it does not
    meet the grid's own edge.  Terms beyond a crop edge count as zero, like terms beyond the grid (the
    out-of-range rule of section 2.2), and can reach only cells within the dependence radius of that edge,
    so on the sampled region the crop gives the full grid's result.  Returns (window of the oracle result,
    (row slice, column slice) of the sampled region in full-grid indices)."""
    R = dependence_radius(w, p, steps)
    nz, nr = w.nz[p], w.nr[p]
    a, b = max(0, zc - half), min(nz, zc + half)
    z0, z1 = max(0, a - R), min(nz, b + R)
    kmax = min(kmax, nr)
    kr = min(nr, kmax + R)
    g = oracle.Grid(nz=z1 - z0, nr=kr, m=w.m[p], fd_order=w.fd_order[p], taylor_order=w.taylor_order,
                    dz=w.dz, dr=w.dr, dt=w.dt, k0=w.k0)
    psi = np.ascontiguousarray(psi0[:, :kr, z0:z1])
    jj = None if J is None else np.ascontiguousarray(J[..., :kr, z0:z1])
    out = oracle.step(g, psi, jj, steps)
    return out[:, :kmax, a - z0:b - z0], (slice(0, kmax), slice(a, b))
