"""Plain CPU FP64 oracle of the FDETD field update and the envelope propagator (arXiv 2605.12132).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package; the product package never does.  The C source (``fdetd_oracle.c``) is built
with ``gcc -O2 -ffp-contract=off -fopenmp`` into ``oracle/_build/liboracle.so``.

Arrays follow the documented storage: a plane is ``[nr, nz]`` complex128 (z fastest); a Maxwell state
is ``[6, nr, nz]`` (E_rho, E_theta, E_z, B_rho, B_theta, B_z); a current is ``[3, nr, nz]``
(J_rho, J_theta, J_z); the envelope uses planes ``a``, ``a_tilde`` and a real ``chi``.

Every function in this module only marshals arguments; the arithmetic is in the C file, each function
of which cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdetd_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

OP_DZ_MINUS, OP_DZ_PLUS, OP_DR_MINUS, OP_DR_PLUS, OP_DIV_MINUS, OP_DIV_PLUS = 0, 1, 2, 3, 4, 5
OP_SHIFT_MINUS, OP_LAP_RHO, OP_LAP_Z, OP_DZ_CENTRED, OP_AXIS = 6, 7, 8, 9, 10
OP_SHIFT_PLUS_RHO, OP_SHIFT_PLUS_Z = 11, 12


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP over rows)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                        "-fPIC", "-shared", "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [("nz", C.c_int32), ("nr", C.c_int32), ("m", C.c_int32), ("fd_order", C.c_int32),
                ("taylor_order", C.c_int32), ("pad_", C.c_int32),
                ("dz", C.c_double), ("dr", C.c_double), ("dt", C.c_double), ("k0", C.c_double)]


@dataclass
class Grid:
    """One problem: grid sizes, mode, orders and steps (normalised units, c = 1)."""
    nz: int
    nr: int
    m: int
    fd_order: int
    taylor_order: int
    dz: float
    dr: float
    dt: float
    k0: float = 1.0

    def c(self) -> Problem:
        return Problem(self.nz, self.nr, self.m, self.fd_order, self.taylor_order, 0,
                       self.dz, self.dr, self.dt, self.k0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER(Problem)
        vp = C.c_void_p
        for name in ("oracle_coef_staggered", "oracle_coef_halfshift", "oracle_coef_centred_d1",
                     "oracle_coef_centred_d2", "oracle_coef_axis"):
            getattr(L, name).argtypes = [C.c_int, vp]
            getattr(L, name).restype = None
        L.oracle_apply_op.argtypes = [P, C.c_int, C.c_int, C.c_int, vp, vp]
        L.oracle_apply_H.argtypes = [P, vp, vp]
        L.oracle_stage_current.argtypes = [P, vp, vp]
        L.oracle_set_axis.argtypes = [P, vp]
        L.oracle_step.argtypes = [P, vp, vp, C.c_int64, C.c_int]
        L.oracle_step_corrected.argtypes = [P, vp, vp, C.c_int64, C.c_int]
        L.oracle_correct_current.argtypes = [P, vp, vp]
        L.oracle_apply_Ha.argtypes = [P, vp, vp, vp, vp, vp]
        L.oracle_envelope_step.argtypes = [P, vp, vp, vp, C.c_int]
        L.oracle_ponderomotive.argtypes = [P, vp, vp]
        L.oracle_absorber_profile.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double, vp]
        L.oracle_envelope_step_absorbing.argtypes = [P, vp, vp, vp, vp, C.c_int]
        L.oracle_energy.argtypes = [P, vp, vp, vp]
        L.oracle_energy.restype = None
        L.oracle_envelope_energy.argtypes = [P, vp, vp, vp, vp]
        L.oracle_envelope_energy.restype = None
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_set_num_threads.restype = None
        L.oracle_deposit_rho.argtypes = [P, vp, C.c_long, C.c_double, C.c_double, vp]
        L.oracle_deposit_jz.argtypes = [P, vp, C.c_long, C.c_double, C.c_double, vp]
        L.oracle_deposit_current.argtypes = [P, vp, C.c_long, C.c_double, vp, vp]
        L.oracle_destagger.argtypes = [P, vp, vp]
        L.oracle_interpolate.argtypes = [P, vp, vp, C.c_long, vp]
        L.oracle_gather_fine.argtypes = [P, vp, vp, C.c_long, C.c_int, vp]
        L.oracle_envelope_gather.argtypes = [P, vp, vp, C.c_long, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


def _chk(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def _cplx(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.shape == shape, (a.shape, shape)
    return a


def coef(kind: str, nd: int) -> np.ndarray:
    """kind in {'staggered', 'halfshift', 'd1', 'd2', 'axis'}; 'd2' returns [b_0, b_1..b_nd]."""
    n = nd + 1 if kind == "d2" else nd
    out = np.zeros(n, dtype=np.float64)
    fn = {"staggered": "oracle_coef_staggered", "halfshift": "oracle_coef_halfshift",
          "d1": "oracle_coef_centred_d1", "d2": "oracle_coef_centred_d2",
          "axis": "oracle_coef_axis"}[kind]
    getattr(lib(), fn)(nd, _ptr(out))
    return out


def apply_op(g: Grid, op: int, plane, parity: int = 1, axis_extrapolate: bool = False) -> np.ndarray:
    x = _cplx(plane, (g.nr, g.nz))
    out = np.zeros_like(x)
    P = g.c()
    _chk(lib().oracle_apply_op(C.byref(P), op, parity, int(axis_extrapolate), _ptr(x), _ptr(out)), "op")
    return out


def apply_H(g: Grid, v) -> np.ndarray:
    x = _cplx(v, (6, g.nr, g.nz))
    out = np.zeros_like(x)
    P = g.c()
    _chk(lib().oracle_apply_H(C.byref(P), _ptr(x), _ptr(out)), "apply_H")
    return out


def stage_current(g: Grid, j) -> np.ndarray:
    x = _cplx(j, (3, g.nr, g.nz))
    out = np.zeros_like(x)
    P = g.c()
    _chk(lib().oracle_stage_current(C.byref(P), _ptr(x), _ptr(out)), "stage_current")
    return out


def _samples(samples) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64))
    if x.ndim != 2 or x.shape[1] != 4:
        raise ValueError("samples: [n, 4] array of (z, x, y, q w)")
    return x


def deposit_rho(g: Grid, samples, dz_shift: float = 0.0, eps: float = 0.5) -> np.ndarray:
    """Charge density of mode g.m of the samples shifted by dz_shift along z, [nr, nz] complex."""
    x = _samples(samples)
    out = np.zeros((g.nr, g.nz), np.complex128)
    P = g.c()
    _chk(lib().oracle_deposit_rho(C.byref(P), _ptr(x), x.shape[0], dz_shift, eps, _ptr(out)), "deposit_rho")
    return out


def deposit_jz(g: Grid, samples, vz: float = 1.0, eps: float = 0.5, j=None) -> np.ndarray:
    """Longitudinal current of the samples moving with vz, added into plane 2 of j ([3, nr, nz], zeros
    when None); returns j."""
    x = _samples(samples)
    out = np.zeros((3, g.nr, g.nz), np.complex128) if j is None else _cplx(j, (3, g.nr, g.nz)).copy()
    P = g.c()
    _chk(lib().oracle_deposit_jz(C.byref(P), _ptr(x), x.shape[0], vz, eps, _ptr(out)), "deposit_jz")
    return out


def deposit_current(g: Grid, samples, eps: float = 0.5):
    """Currents of moving samples ([n, 8]: z, x, y, q w, v_x, v_y, v_z, unused): returns (j [3, nr, nz],
    rho_xy [nr, nz])."""
    x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64))
    if x.ndim != 2 or x.shape[1] != 8:
        raise ValueError("samples: [n, 8] array of (z, x, y, q w, v_x, v_y, v_z, unused)")
    j = np.zeros((3, g.nr, g.nz), np.complex128)
    r = np.zeros((g.nr, g.nz), np.complex128)
    P = g.c()
    _chk(lib().oracle_deposit_current(C.byref(P), _ptr(x), x.shape[0], eps, _ptr(j), _ptr(r)), "deposit_current")
    return j, r


def set_axis(g: Grid, psi) -> np.ndarray:
    x = _cplx(psi, (6, g.nr, g.nz)).copy()
    P = g.c()
    _chk(lib().oracle_set_axis(C.byref(P), _ptr(x)), "set_axis")
    return x


def step(g: Grid, psi, j=None, n_steps: int = 1) -> np.ndarray:
    """Advance a copy of psi by n_steps.  j is None, one [3,nr,nz] block used every step, or
    [n_steps,3,nr,nz] with one block per step."""
    x = _cplx(psi, (6, g.nr, g.nz)).copy()
    stride = 0
    jj = None
    if j is not None:
        jj = np.ascontiguousarray(j, dtype=np.complex128)
        if jj.ndim == 4:
            assert jj.shape[0] >= n_steps and jj.shape[1:] == (3, g.nr, g.nz)
            stride = 3 * g.nr * g.nz
        else:
            assert jj.shape == (3, g.nr, g.nz)
    P = g.c()
    _chk(lib().oracle_step(C.byref(P), _ptr(x), _ptr(jj), stride, n_steps), "step")
    return x


def apply_Ha(g: Grid, a, at, chi):
    a = _cplx(a, (g.nr, g.nz))
    at = _cplx(at, (g.nr, g.nz))
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    assert chi.shape == (g.nr, g.nz)
    oa, ot = np.zeros_like(a), np.zeros_like(at)
    P = g.c()
    _chk(lib().oracle_apply_Ha(C.byref(P), _ptr(a), _ptr(at), _ptr(chi), _ptr(oa), _ptr(ot)), "apply_Ha")
    return oa, ot


def envelope_step(g: Grid, a, at, chi, n_steps: int = 1):
    a = _cplx(a, (g.nr, g.nz)).copy()
    at = _cplx(at, (g.nr, g.nz)).copy()
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    assert chi.shape == (g.nr, g.nz)
    P = g.c()
    _chk(lib().oracle_envelope_step(C.byref(P), _ptr(a), _ptr(at), _ptr(chi), n_steps), "envelope_step")
    return a, at


def ponderomotive(g: Grid, a):
    """|a|^2, A~_rho = -D_rho^(-)|a|^2, A~_z = -D_z^(-)|a|^2 of an m = 0 envelope: [3, nr, nz] real."""
    x = _cplx(a, (g.nr, g.nz))
    out = np.zeros((3, g.nr, g.nz))
    P = g.c()
    _chk(lib().oracle_ponderomotive(C.byref(P), _ptr(x), _ptr(out)), "ponderomotive")
    return out


def envelope_gather(g: Grid, pond, samples):
    """|a|^2, A~_rho, A~_z of an m = 0 envelope ([3, nr, nz] real, as `ponderomotive` returns) at the
    samples ([n, 4]: z, x, y, unused) (section 4.3): [n, 3] doubles."""
    x = np.ascontiguousarray(pond, dtype=np.float64)
    assert x.shape == (3, g.nr, g.nz)
    s = np.ascontiguousarray(samples, dtype=np.float64)
    assert s.ndim == 2 and s.shape[1] == 4
    out = np.zeros((s.shape[0], 3))
    P = g.c()
    _chk(lib().oracle_envelope_gather(C.byref(P), _ptr(x), _ptr(s), s.shape[0], _ptr(out)), "envelope_gather")
    return out


def absorber_profile(g: Grid, lz: int, lr: int, sigma_max: float, power: float = 2.0):
    """Layer functions sigma [nr][nz] of the scalar absorbing layer (polynomial grading: a reading, since the paper leaves the layer functions to a companion paper)."""
    sigma = np.zeros((g.nr, g.nz))
    P = g.c()
    _chk(lib().oracle_absorber_profile(C.byref(P), lz, lr, sigma_max, power, _ptr(sigma)), "absorber_profile")
    return sigma


def envelope_step_absorbing(g: Grid, a, at, chi, sigma, n_steps: int = 1):
    """n_steps of exp(-sigma dt/4) T_N(dt H_a(chi + sigma^2)) exp(-sigma dt/4) on (a, a_tilde)."""
    a = _cplx(a, (g.nr, g.nz)).copy()
    at = _cplx(at, (g.nr, g.nz)).copy()
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    assert chi.shape == (g.nr, g.nz) and sigma.shape == (g.nr, g.nz)
    P = g.c()
    _chk(lib().oracle_envelope_step_absorbing(C.byref(P), _ptr(a), _ptr(at), _ptr(chi), _ptr(sigma), n_steps),
         "envelope_step_absorbing")
    return a, at


def energy(g: Grid, psi):
    x = _cplx(psi, (6, g.nr, g.nz))
    e, z = C.c_double(), C.c_double()
    P = g.c()
    lib().oracle_energy(C.byref(P), _ptr(x), C.byref(e), C.byref(z))
    return e.value, z.value


def envelope_energy(g: Grid, a, at):
    a = _cplx(a, (g.nr, g.nz))
    at = _cplx(at, (g.nr, g.nz))
    e, z = C.c_double(), C.c_double()
    P = g.c()
    lib().oracle_envelope_energy(C.byref(P), _ptr(a), _ptr(at), C.byref(e), C.byref(z))
    return e.value, z.value


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_num_threads(int(n))


def destagger(g: Grid, psi):
    """The six components of a state on the primary grids (section 3.3), [6, nr, nz]."""
    x = _cplx(psi, (6, g.nr, g.nz))
    out = np.zeros_like(x)
    P = g.c()
    _chk(lib().oracle_destagger(C.byref(P), _ptr(x), _ptr(out)), "destagger")
    return out


def interpolate(g: Grid, prim, samples):
    """Mode g.m of six primary-grid planes [6, nr, nz] at the samples: [n, 6] doubles (section 3.3)."""
    x = _cplx(prim, (6, g.nr, g.nz))
    s = np.ascontiguousarray(samples, dtype=np.float64)
    out = np.zeros((s.shape[0], 6))
    P = g.c()
    _chk(lib().oracle_interpolate(C.byref(P), _ptr(x), _ptr(s), s.shape[0], _ptr(out)), "interpolate")
    return out


def gather(grids, states, samples):
    """Fields at the samples: for every (grid, state) pair (the modes of one grid), the destaggered
    components interpolated with cubic shapes and summed as Re(F_m e^(i m theta)); [n, 6] doubles
    (E_rho, E_theta, E_z, B_rho, B_theta, B_z)."""
    s = np.ascontiguousarray(samples, dtype=np.float64)
    assert s.ndim == 2 and s.shape[1] == 4
    out = np.zeros((s.shape[0], 6))
    for g, psi in zip(grids, states):
        prim = destagger(g, psi)
        P = g.c()
        _chk(lib().oracle_interpolate(C.byref(P), _ptr(prim), _ptr(s), s.shape[0], _ptr(out)), "interpolate")
    return out


def gather_fine(grids, states, samples, supersample: int):
    """Fields at the samples with the resolution doubled before the shape sum (section 3.4): supersample
    bit 0 along z, bit 1 along rho (0 gives the plain gather); [n, 6] doubles, summed over the modes."""
    s = np.ascontiguousarray(samples, dtype=np.float64)
    assert s.ndim == 2 and s.shape[1] == 4
    out = np.zeros((s.shape[0], 6))
    for g, psi in zip(grids, states):
        x = _cplx(psi, (6, g.nr, g.nz))
        P = g.c()
        _chk(lib().oracle_gather_fine(C.byref(P), _ptr(x), _ptr(s), s.shape[0], int(supersample), _ptr(out)),
             "gather_fine")
    return out


def correct_current(g: Grid, jbar, rho_xy):
    """Current correction of section 3.7 on a staged current [3, nr, nz] (J_rho staggered) with the planar
    density differential rho_xy [nr, nz]; returns the corrected current."""
    x = _cplx(jbar, (3, g.nr, g.nz)).copy()
    r = _cplx(rho_xy, (g.nr, g.nz))
    P = g.c()
    _chk(lib().oracle_correct_current(C.byref(P), _ptr(x), _ptr(r)), "correct_current")
    return x


def step_corrected(g: Grid, psi, j4, n_steps: int = 1):
    """n_steps with the current correction: j4 is [4, nr, nz] (the same block every step) or
    [n_steps, 4, nr, nz] (J_rho, J_theta, J_z, rho_xy)."""
    psi = _cplx(psi, (6, g.nr, g.nz)).copy()
    j = np.ascontiguousarray(j4, dtype=np.complex128)
    stride = 0 if j.ndim == 3 else 4 * g.nr * g.nz
    P = g.c()
    _chk(lib().oracle_step_corrected(C.byref(P), _ptr(psi), _ptr(j), stride, n_steps), "step_corrected")
    return psi
