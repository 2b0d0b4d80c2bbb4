"""Float accumulation schemes for the Taylor propagator, emulated on the CPU (float32 numpy; H applied by the
oracle in FP64 and rounded to float, so each H application carries one float rounding), against the FP64
oracle.  This is a model of the FP32C design choice, not a parity test of the GPU path.

Schemes, each one step of the exponential solution with the midpoint source (section 2.1, Taylor sum of
section 2.5), state stored as a float pair (hi, lo) where compensated:
  * plain:  Horner in float, v_n = fl(w_n + c_n H v_{n+1}), w_n = hi + beta_n Jbar, new hi = fl(hi + inc);
  * twosum: the same Horner, the last addition done as TwoSum(hi, lo + inc) (the library's FP32C today);
  * kahan:  the two forward series of the exponential, p_n = (dt/n) H p_{n-1} from psi and q_n =
            (dt/2n) H q_{n-1} from Jbar, every term added into (S, c) by Kahan's compensated summation;
  * increment: Horner on the increment d_n = v_n - psi: d_N = beta_N Jbar,
            d_n = beta_n Jbar + c_n (P + H d_{n+1}) with P = H hi + H lo formed once per step, then
            TwoSum(hi, lo + d_0).  The stage vectors are of the increment's size, not of psi's.

On grid-scale random fields (the largest ||dt H||) every scheme lands within 15 % of the others.  On
resolved pulses the Horner intermediates of plain and twosum are rounded at the scale of psi, and that
rounding reaches the state through dt H at full weight each step, so their compensation buys nothing;
the literal series and, more so, the increment form keep every rounding at the scale of the terms."""
import numpy as np
import pytest

from helpers import grid_of, rel_l2, tol_fp32c

import oracle
import paper_2605_12132_amd.inputs as I


def f32(x):
    return np.asarray(x, dtype=np.complex128).astype(np.complex64)


def two_sum(a, b):
    s = f32(a + b)
    bb = f32(s - a)
    return s, f32(f32(a - f32(s - bb)) + f32(b - bb))


def Hf(g, v):
    return f32(oracle.apply_H(g, np.asarray(v, dtype=np.complex128)))


def run(g, psi0, J, steps, scheme):
    N, dt = g.taylor_order, g.dt
    hi, lo = f32(psi0), f32(np.zeros_like(psi0))
    for s in range(steps):
        jb = np.zeros_like(hi)
        jb[:3] = f32(oracle.stage_current(g, J[s]))
        if scheme in ("plain", "twosum"):
            v = f32(hi + f32(-dt * 2.0 ** -N * jb))
            for n in range(N - 1, -1, -1):
                inc = f32(f32(-dt * 2.0 ** -n * jb) + f32((dt / (n + 1)) * Hf(g, v).astype(np.complex128)))
                if n > 0:
                    v = f32(hi + inc)
                elif scheme == "twosum":
                    hi, lo = two_sum(hi, f32(lo + inc))
                else:
                    hi = f32(hi + inc)
        elif scheme == "increment":
            P = f32(Hf(g, hi) + Hf(g, lo))
            d = f32(-dt * 2.0 ** -N * jb)
            for n in range(N - 1, -1, -1):
                d = f32(f32(-dt * 2.0 ** -n * jb) + f32((dt / (n + 1)) * f32(P + Hf(g, d)).astype(np.complex128)))
            hi, lo = two_sum(hi, f32(lo + d))
        else:  # literal Kahan summation of the series terms, compensation carried across steps in lo
            S, c = hi, f32(-lo)

            def kadd(S, c, x):
                y = f32(x - c)
                t = f32(S + y)
                return t, f32(f32(t - S) - y)
            p, q = hi, jb
            S, c = kadd(S, c, f32(-dt * jb))
            for n in range(1, N + 1):
                p = f32((dt / n) * Hf(g, p).astype(np.complex128))
                q = f32((0.5 * dt / n) * Hf(g, q).astype(np.complex128))
                S, c = kadd(S, c, p)
                S, c = kadd(S, c, f32(-dt * q))
            hi, lo = S, f32(-c)
        # axis slots derived on output (section 2.4), from both words of the state
        tot = oracle.set_axis(g, hi.astype(np.complex128) + lo.astype(np.complex128))
        hi = f32(tot)
        lo = f32(tot - hi)
    return hi.astype(np.complex128) + lo.astype(np.complex128)


SCHEMES = ("plain", "twosum", "kahan", "increment")


def errors(g, psi0, J, steps):
    ref = oracle.step(g, psi0, J, steps)
    return {s: rel_l2(run(g, psi0, J, steps, s), ref) for s in SCHEMES}


def test_emulation_is_the_oracle_step_in_exact_arithmetic(monkeypatch):
    """With the float rounding switched off every scheme is the oracle's step (to FP64 rounding)."""
    import sys
    mod = sys.modules[__name__]
    monkeypatch.setattr(mod, "f32", lambda x: np.asarray(x, dtype=np.complex128))
    dz = I.LAMBDA0 / 20
    g = oracle.Grid(nz=64, nr=24, m=1, fd_order=8, taylor_order=8, dz=dz, dr=2 * dz, dt=0.5 * dz, k0=1.0)
    rng = np.random.default_rng(3)
    psi0 = rng.uniform(-1, 1, (6, 24, 64)) + 1j * rng.uniform(-1, 1, (6, 24, 64))
    J = 0.1 * (rng.uniform(-1, 1, (3, 3, 24, 64)) + 1j * rng.uniform(-1, 1, (3, 3, 24, 64)))
    ref = oracle.step(g, psi0, J, 3)
    for s in SCHEMES:
        assert rel_l2(run(g, psi0, J, 3, s), ref) < 1e-13, s


def test_random_fields_all_schemes_alike():
    dz = I.LAMBDA0 / 20
    g = oracle.Grid(nz=96, nr=40, m=1, fd_order=16, taylor_order=8, dz=dz, dr=2 * dz, dt=0.5 * dz, k0=1.0)
    rng = np.random.default_rng(7)
    psi0 = rng.uniform(-1, 1, (6, 40, 96)) + 1j * rng.uniform(-1, 1, (6, 40, 96))
    J = 0.1 * (rng.uniform(-1, 1, (40, 3, 40, 96)) + 1j * rng.uniform(-1, 1, (40, 3, 40, 96)))
    e = errors(g, psi0, J, 40)
    print("random fields, 40 steps:", {k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) < 1.15 * min(e.values())
    assert max(e.values()) < tol_fp32c(40, 8)


@pytest.mark.parametrize("name", ["vacuum pulse", "current-driven"])
def test_resolved_pulse_increment_form_is_the_most_accurate(name):
    if name == "vacuum pulse":
        w = I.vacuum_pulse()
        steps = 100
        J = np.zeros((steps, 3, w.nr[0], w.nz[0]), complex)
    else:
        w = I.current_driven().shrink(nz=400, nr=48)
        steps = 100
        J = I.currents(w, 0, steps)
    g = grid_of(w, 0)
    e = errors(g, I.initial_fields(w, 0), J, steps)
    print(f"{name}, {steps} steps:", {k: f"{v:.2e}" for k, v in e.items()})
    assert e["twosum"] < tol_fp32c(steps, w.taylor_order)
    assert e["twosum"] > 0.7 * e["plain"]          # the final TwoSum alone buys little here
    assert e["kahan"] < 0.8 * e["twosum"]
    assert e["increment"] < 0.5 * e["twosum"] and e["increment"] < e["kahan"]
