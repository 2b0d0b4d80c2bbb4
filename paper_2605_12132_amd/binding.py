"""ctypes binding of the FDETD C-ABI (include/fdetd.h).

Argument marshalling only: every operation runs in the HIP kernels of libfdetd.so.  The functions keep
the C names (fdetd_plan, fdetd_step, envelope_step, ...); ``Plan`` is a small convenience wrapper that
takes PyTorch device tensors and enqueues on torch's current stream.  If the library is missing the
import of this module raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libfdetd.so")

FDETD_OK, FDETD_E_ARG, FDETD_E_UNSTABLE, FDETD_E_NOMEM, FDETD_E_HIP = 0, -1, -2, -3, -4
FP64, FP32C = 0, 1
MAXWELL, ENVELOPE = 0, 1
PLAN_SKIP_STABILITY, PLAN_USE_GRAPH, PLAN_PROFILE, PLAN_NO_AUTOTUNE, PLAN_ONE_STREAM = 1, 2, 4, 8, 16
PLAN_CURRENT_CORRECTION = 32
PLAN_MIXED_WIDTHS = 64
PLAN_PER_WIDTH = 128
PLAN_INCREMENT_FORM = 256
PLAN_SEPARATE_WN = 512

# every symbol declared in include/fdetd.h
EXPORTS = ("fdetd_plan", "fdetd_step", "fdetd_step_graph", "fdetd_step_noalloc", "envelope_step", "envelope_absorber", "envelope_ponderomotive",
           "envelope_gather",
           "fdetd_deposit_jz", "fdetd_deposit_rho",
           "fdetd_deposit_current", "fdetd_gather", "fdetd_gather_supersampled", "fdetd_query",
           "fdetd_export_state",
           "fdetd_import_state", "fdetd_coefficients", "fdetd_taylor_stability_bound", "fdetd_last_error",
           "fdetd_destroy")


class FdetdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"FDETD error {code}: {msg}")
        self.code = code


class ProblemDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nz", C.c_int32), ("nr", C.c_int32), ("m", C.c_int32),
                ("fd_order", C.c_int32), ("taylor_order", C.c_int32),
                ("dz", C.c_double), ("dr", C.c_double), ("dt", C.c_double), ("k0", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("n_probs", C.c_int32), ("precision", C.c_int32), ("dt_rho_max", C.c_double),
                ("stability_margin", C.c_double), ("cells", C.c_int64), ("bytes_per_step", C.c_int64),
                ("scratch_bytes", C.c_int64), ("launches_per_step", C.c_int64),
                ("profiled_launches", C.c_int64), ("profiled_ms", C.c_double), ("profiled_bytes", C.c_double),
                ("seg_rows", C.c_int32), ("seg_rows_axis", C.c_int32), ("autotune_ms", C.c_double),
                ("streams", C.c_int32), ("store_policy", C.c_int32), ("tile_order", C.c_int32)]


JGEN_BUNCH, JGEN_SAMPLES = 1, 2


class JgenDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("step0", C.c_int64), ("seed", C.c_uint64),
                ("nb", C.c_double), ("sigz", C.c_double), ("sigr", C.c_double), ("z0_frac", C.c_double),
                ("vb", C.c_double), ("noise", C.c_double), ("samples", C.c_void_p), ("n", C.c_int64),
                ("vz", C.c_double), ("eps", C.c_double)]


@dataclass
class Jgen:
    """In-graph current of fdetd_step_graph: kind JGEN_BUNCH (bunch + SplitMix64 noise) or JGEN_SAMPLES
    (a float64 [n, 4] cuda tensor of samples (z at t = 0, x, y, q w) moving with vz, deposited each step)."""
    kind: int
    step0: int = 0
    seed: int = 0
    nb: float = 0.0
    sigz: float = 0.0
    sigr: float = 0.0
    z0_frac: float = 0.25
    vb: float = 1.0
    noise: float = 0.0
    samples: object = None
    vz: float = 1.0
    eps: float = 0.5

    def c(self) -> JgenDesc:
        ptr, n = 0, 0
        if self.samples is not None:
            import torch
            x = self.samples
            if not (x.is_cuda and x.dtype == torch.float64 and x.dim() == 2 and x.shape[1] == 4 and x.is_contiguous()):
                raise ValueError("samples: contiguous float64 cuda tensor [n, 4]")
            ptr, n = x.data_ptr(), x.shape[0]
        return JgenDesc(self.kind, 0, self.step0, self.seed % 2 ** 64, self.nb, self.sigz, self.sigr, self.z0_frac,
                        self.vb, self.noise, ptr, n, self.vz, self.eps)


@dataclass
class Problem:
    """One grid and one azimuthal mode (normalised units, c = 1)."""
    nz: int
    nr: int
    m: int
    fd_order: int
    taylor_order: int
    dz: float
    dr: float
    dt: float
    k0: float = 1.0
    kind: int = MAXWELL

    def c(self) -> ProblemDesc:
        return ProblemDesc(self.kind, self.nz, self.nr, self.m, self.fd_order, self.taylor_order,
                           self.dz, self.dr, self.dt, self.k0)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run paper_2605_12132_amd/build.py (hipcc, gfx950)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 / libhsa-runtime64.so.1.  Loading
    # torch first makes the library's dependencies resolve (by soname) to the copies torch already mapped,
    # so device memory, streams and kernels all live in the same runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, pp = C.c_void_p, C.POINTER(C.c_void_p)
    L.fdetd_plan.argtypes = [C.POINTER(ProblemDesc), C.c_int32, C.c_int32, C.c_uint32, vp, C.POINTER(vp)]
    L.fdetd_step.argtypes = [vp, pp, pp, C.c_int64, C.c_int32]
    L.envelope_step.argtypes = [vp, pp, pp, pp, C.c_int64, C.c_int32]
    L.fdetd_step_graph.argtypes = [vp, pp, C.POINTER(JgenDesc), pp, C.c_int32]
    L.fdetd_step_noalloc.argtypes = [C.POINTER(ProblemDesc), C.c_int32, vp, vp, vp, C.c_int64, C.c_int32]
    L.fdetd_deposit_jz.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_double, pp]
    L.fdetd_deposit_rho.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_double, pp]
    L.fdetd_gather.argtypes = [vp, pp, vp, C.c_int64, vp]
    L.fdetd_gather_supersampled.argtypes = [vp, pp, vp, C.c_int64, vp, C.c_int32]
    L.envelope_gather.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, vp]
    L.envelope_ponderomotive.argtypes = [vp, pp, pp]
    L.fdetd_deposit_current.argtypes = [vp, vp, C.c_int64, C.c_double, pp]
    L.envelope_absorber.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double]
    L.fdetd_query.argtypes = [vp, C.POINTER(PlanInfo)]
    L.fdetd_export_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.fdetd_import_state.argtypes = [vp, vp, C.c_size_t]
    L.fdetd_coefficients.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.fdetd_taylor_stability_bound.argtypes = [C.c_int32]
    L.fdetd_taylor_stability_bound.restype = C.c_double
    L.fdetd_last_error.argtypes = [vp]
    L.fdetd_last_error.restype = C.c_char_p
    L.fdetd_destroy.argtypes = [vp]
    L.fdetd_destroy.restype = None
    return L


lib = _load()


def fdetd_last_error(plan=None) -> str:
    s = lib.fdetd_last_error(plan)
    return s.decode() if s else ""


def _check(rc: int, plan=None):
    if rc != FDETD_OK:
        raise FdetdError(rc, fdetd_last_error(plan))


def _ptrs(xs) -> C.Array:
    arr = (C.c_void_p * len(xs))()
    for i, x in enumerate(xs):
        arr[i] = x
    return arr


def fdetd_plan(problems: Sequence[Problem], precision: int = FP64, flags: int = 0, stream: int = 0):
    descs = (ProblemDesc * len(problems))(*[p.c() for p in problems])
    out = C.c_void_p()
    rc = lib.fdetd_plan(descs, len(problems), precision, flags, C.c_void_p(stream), C.byref(out))
    _check(rc, None)
    return out.value


def fdetd_step(plan, psi_ptrs, j_ptrs=None, j_step_blocks: int = 0, n_steps: int = 1):
    rc = lib.fdetd_step(plan, _ptrs(psi_ptrs), _ptrs(j_ptrs) if j_ptrs is not None else None,
                        j_step_blocks, n_steps)
    _check(rc, plan)


def fdetd_step_graph(plan, psi_ptrs, jgen: "JgenDesc | None", jw_ptrs, n_steps: int):
    rc = lib.fdetd_step_graph(plan, _ptrs(psi_ptrs), C.byref(jgen) if jgen is not None else None,
                              _ptrs(jw_ptrs) if jw_ptrs is not None else None, n_steps)
    _check(rc, plan)


def fdetd_step_noalloc(problem: Problem, precision: int, stream: int, psi_ptr: int, j_ptr=None,
                       j_step_blocks: int = 0, n_steps: int = 1):
    """fdetd_step of one Maxwell problem without a plan and without device allocation (raw pointers)."""
    d = problem.c()
    rc = lib.fdetd_step_noalloc(C.byref(d), precision, C.c_void_p(stream), C.c_void_p(psi_ptr),
                                C.c_void_p(j_ptr) if j_ptr is not None else None, j_step_blocks, n_steps)
    _check(rc, None)


def envelope_step(plan, a_ptrs, at_ptrs, chi_ptrs, chi_step_planes: int = 0, n_steps: int = 1):
    rc = lib.envelope_step(plan, _ptrs(a_ptrs), _ptrs(at_ptrs), _ptrs(chi_ptrs), chi_step_planes, n_steps)
    _check(rc, plan)


def fdetd_deposit_jz(plan, samples_ptr, n: int, vz: float, eps: float, j_ptrs):
    rc = lib.fdetd_deposit_jz(plan, samples_ptr, n, vz, eps, _ptrs(j_ptrs))
    _check(rc, plan)


def fdetd_deposit_rho(plan, samples_ptr, n: int, dz_shift: float, eps: float, rho_ptrs):
    _check(lib.fdetd_deposit_rho(plan, samples_ptr, n, dz_shift, eps, _ptrs(rho_ptrs)), plan)


def fdetd_deposit_current(plan, samples_ptr, n: int, eps: float, j_ptrs):
    _check(lib.fdetd_deposit_current(plan, samples_ptr, n, eps, _ptrs(j_ptrs)), plan)


def envelope_ponderomotive(plan, a_ptrs, out_ptrs):
    _check(lib.envelope_ponderomotive(plan, _ptrs(a_ptrs), _ptrs(out_ptrs)), plan)


def fdetd_gather(plan, psi_ptrs, samples_ptr, n: int, fields_ptr):
    _check(lib.fdetd_gather(plan, _ptrs(psi_ptrs), samples_ptr, n, fields_ptr), plan)


def fdetd_gather_supersampled(plan, psi_ptrs, samples_ptr, n: int, fields_ptr, supersample: int):
    _check(lib.fdetd_gather_supersampled(plan, _ptrs(psi_ptrs), samples_ptr, n, fields_ptr, supersample), plan)


def envelope_gather(plan, problem: int, pond_ptr, samples_ptr, n: int, out_ptr):
    _check(lib.envelope_gather(plan, problem, pond_ptr, samples_ptr, n, out_ptr), plan)


def envelope_absorber(plan, problem: int, lz: int, lr: int, sigma_max: float, power: float = 2.0):
    _check(lib.envelope_absorber(plan, problem, lz, lr, sigma_max, power), plan)


def fdetd_query(plan) -> dict:
    info = PlanInfo()
    _check(lib.fdetd_query(plan, C.byref(info)), plan)
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def fdetd_export_state(plan) -> bytes:
    n = C.c_size_t(0)
    _check(lib.fdetd_export_state(plan, None, C.byref(n)), plan)
    buf = C.create_string_buffer(max(n.value, 1))
    _check(lib.fdetd_export_state(plan, buf, C.byref(n)), plan)
    return buf.raw[:n.value]


def fdetd_import_state(plan, blob: bytes):
    _check(lib.fdetd_import_state(plan, blob if blob else None, len(blob)), plan)


def fdetd_coefficients(which: int, nd: int):
    out = (C.c_double * (nd + 1))()
    _check(lib.fdetd_coefficients(which, nd, out), None)
    n = nd + 1 if which == 3 else nd
    return [out[i] for i in range(n)]


def fdetd_taylor_stability_bound(n: int) -> float:
    return float(lib.fdetd_taylor_stability_bound(n))


def fdetd_destroy(plan):
    lib.fdetd_destroy(plan)


class Plan:
    """Owns one fdetd plan bound to torch's current CUDA (HIP) stream at construction."""

    def __init__(self, problems: Sequence[Problem], precision: int = FP64, flags: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("FDETD needs a gfx950 GPU; none is visible")
        self.problems = list(problems)
        self.precision = precision
        self.flags = flags
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = fdetd_plan(self.problems, precision, flags, self.stream.cuda_stream)

    # --- tensor checks (shape / dtype / device / contiguity), then raw pointers ---
    def _cdtype(self):
        import torch
        return torch.complex128 if self.precision == FP64 else torch.complex64

    def _rdtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    def _nchk(self, xs, what):
        if len(xs) != len(self.problems):
            raise ValueError(f"{what}: {len(xs)} tensors for {len(self.problems)} problems")

    def _chk(self, t, shape_tail, dtype, what):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape[-len(shape_tail):]) != shape_tail:
            raise ValueError(f"{what}: need contiguous {dtype} cuda tensor [..., {shape_tail}], got "
                             f"{t.dtype} {tuple(t.shape)} cuda={t.is_cuda} contiguous={t.is_contiguous()}")
        return t.data_ptr()

    def step(self, psi, j_half=None, n_steps: int = 1):
        """psi: list of [6, nr, nz] tensors; j_half: None, list of [3, nr, nz] (same current every step)
        or [n_steps, 3, nr, nz] (one current per step); 4 planes instead of 3 (J_rho, J_theta, J_z,
        rho_xy) with PLAN_CURRENT_CORRECTION."""
        cd = self._cdtype()
        self._nchk(psi, "psi")
        if j_half is not None:
            self._nchk(j_half, "j_half")
        pp = [self._chk(x, (6, p.nr, p.nz), cd, "psi") for x, p in zip(psi, self.problems)]
        jp, stride = None, 0
        if j_half is not None:
            nb = 4 if self.flags & PLAN_CURRENT_CORRECTION else 3  # J_rho, J_theta, J_z (, rho_xy)
            jp = [self._chk(x, (nb, p.nr, p.nz), cd, "j_half") for x, p in zip(j_half, self.problems)]
            dims = {x.dim() for x in j_half}
            if len(dims) != 1 or dims - {3, 4}:
                raise ValueError("j_half: all [3, nr, nz] or all [steps, 3, nr, nz]")
            if 4 in dims and n_steps > 1:
                if any(x.shape[0] < n_steps for x in j_half):
                    raise ValueError("j_half has fewer steps than n_steps")
                stride = 1
        fdetd_step(self._h, pp, jp, stride, n_steps)

    def step_graph(self, psi, jgen: "Jgen | None", j_work=None, n_steps: int = 1):
        """n_steps steps whose current jgen makes every step into j_work (list of [3, nr, nz] tensors of the
        plan's precision, overwritten); captured as one hipGraph with PLAN_USE_GRAPH."""
        cd = self._cdtype()
        self._nchk(psi, "psi")
        pp = [self._chk(x, (6, p.nr, p.nz), cd, "psi") for x, p in zip(psi, self.problems)]
        jp = None
        if jgen is not None:
            self._nchk(j_work, "j_work")
            jp = [self._chk(x, (3, p.nr, p.nz), cd, "j_work") for x, p in zip(j_work, self.problems)]
        self._jgen_keep = jgen.c() if jgen is not None else None  # alive while the call reads it
        fdetd_step_graph(self._h, pp, self._jgen_keep, jp, n_steps)

    def deposit_jz(self, samples, j_half, vz: float = 1.0, eps: float = 0.5):
        """Add the longitudinal current of point samples (float64 [n, 4] cuda tensor of z, x, y, q w) into
        plane 2 of each problem's current (list of [3, nr, nz] tensors of the plan's precision)."""
        import torch
        if not (samples.is_cuda and samples.dtype == torch.float64 and samples.dim() == 2 and samples.shape[1] == 4
                and samples.is_contiguous()):
            raise ValueError("samples: contiguous float64 cuda tensor [n, 4]")
        self._nchk(j_half, "j_half")
        jp = [self._chk(x, (3, p.nr, p.nz), self._cdtype(), "j_half") for x, p in zip(j_half, self.problems)]
        fdetd_deposit_jz(self._h, samples.data_ptr(), samples.shape[0], vz, eps, jp)

    def deposit_current(self, samples, j_half, eps: float = 0.5):
        """Add the currents of moving samples (float64 [n, 8] cuda tensor: z, x, y, q w, v_x, v_y, v_z, unused)
        into each problem's current block ([3 or 4, nr, nz] tensors of the plan's precision; plane 3 takes
        rho_xy with PLAN_CURRENT_CORRECTION)."""
        import torch
        if not (samples.is_cuda and samples.dtype == torch.float64 and samples.dim() == 2 and samples.shape[1] == 8
                and samples.is_contiguous()):
            raise ValueError("samples: contiguous float64 cuda tensor [n, 8]")
        self._nchk(j_half, "j_half")
        nb = 4 if self.flags & PLAN_CURRENT_CORRECTION else 3
        jp = [self._chk(x, (nb, p.nr, p.nz), self._cdtype(), "j_half") for x, p in zip(j_half, self.problems)]
        fdetd_deposit_current(self._h, samples.data_ptr(), samples.shape[0], eps, jp)

    def deposit_rho(self, samples, rho, dz_shift: float = 0.0, eps: float = 0.5):
        """Add the charge density of point samples (float64 [n, 4] cuda tensor of z, x, y, q w) shifted by
        dz_shift along z into one plane per problem (list of [nr, nz] tensors of the plan's precision)."""
        import torch
        if not (samples.is_cuda and samples.dtype == torch.float64 and samples.dim() == 2 and samples.shape[1] == 4
                and samples.is_contiguous()):
            raise ValueError("samples: contiguous float64 cuda tensor [n, 4]")
        self._nchk(rho, "rho")
        rp = [self._chk(x, (p.nr, p.nz), self._cdtype(), "rho") for x, p in zip(rho, self.problems)]
        fdetd_deposit_rho(self._h, samples.data_ptr(), samples.shape[0], dz_shift, eps, rp)

    def gather(self, psi, samples, fields=None, supersample: int = 0):
        """Fields (float64 [n, 6] cuda tensor: E_rho, E_theta, E_z, B_rho, B_theta, B_z) at the samples
        (float64 [n, 4] cuda tensor of z, x, y, w) of the plan's modes of one grid; supersample: bit 0
        doubles the resolution along z, bit 1 along rho, before the shape sum."""
        import torch
        if not (samples.is_cuda and samples.dtype == torch.float64 and samples.dim() == 2 and samples.shape[1] == 4
                and samples.is_contiguous()):
            raise ValueError("samples: contiguous float64 cuda tensor [n, 4]")
        self._nchk(psi, "psi")
        pp = [self._chk(x, (6, p.nr, p.nz), self._cdtype(), "psi") for x, p in zip(psi, self.problems)]
        if fields is None:
            fields = torch.empty((samples.shape[0], 6), dtype=torch.float64, device=samples.device)
        if not (fields.is_cuda and fields.dtype == torch.float64 and fields.is_contiguous()
                and tuple(fields.shape) == (samples.shape[0], 6)):
            raise ValueError("fields: contiguous float64 cuda tensor [n, 6]")
        if supersample:
            fdetd_gather_supersampled(self._h, pp, samples.data_ptr(), samples.shape[0], fields.data_ptr(),
                                      int(supersample))
        else:
            fdetd_gather(self._h, pp, samples.data_ptr(), samples.shape[0], fields.data_ptr())
        return fields

    def envelope_step(self, a, a_tilde, chi, n_steps: int = 1):
        cd, rd = self._cdtype(), self._rdtype()
        for x, what in ((a, "a"), (a_tilde, "a_tilde"), (chi, "chi")):
            self._nchk(x, what)
        ap = [self._chk(x, (p.nr, p.nz), cd, "a") for x, p in zip(a, self.problems)]
        tp = [self._chk(x, (p.nr, p.nz), cd, "a_tilde") for x, p in zip(a_tilde, self.problems)]
        cp = [self._chk(x, (p.nr, p.nz), rd, "chi") for x, p in zip(chi, self.problems)]
        stride = 0
        dims = {x.dim() for x in chi}
        if len(dims) != 1 or dims - {2, 3}:
            raise ValueError("chi: all [nr, nz] or all [steps, nr, nz]")
        if 3 in dims and n_steps > 1:
            if any(x.shape[0] < n_steps for x in chi):
                raise ValueError("chi has fewer steps than n_steps")
            stride = 1
        envelope_step(self._h, ap, tp, cp, stride, n_steps)

    def absorber(self, lz: int, lr: int, sigma_max: float, power: float = 2.0, problem: int = -1):
        """Absorbing layers (lz columns at both z ends, lr rows at the outer rho edge, sigma graded as
        sigma_max d^power) for envelope problem `problem`, or all problems (-1)."""
        envelope_absorber(self._h, problem, lz, lr, sigma_max, power)

    def ponderomotive(self, a, out=None):
        """|a|^2, A~_rho, A~_z of the plan's m = 0 envelope problems: list of [3, nr, nz] real tensors."""
        import torch
        self._nchk(a, "a")
        ap = [self._chk(x, (p.nr, p.nz), self._cdtype(), "a") for x, p in zip(a, self.problems)]
        if out is None:
            out = [torch.empty((3, p.nr, p.nz), dtype=self._rdtype(), device=x.device) for x, p in zip(a, self.problems)]
        op = [self._chk(x, (3, p.nr, p.nz), self._rdtype(), "out") for x, p in zip(out, self.problems)]
        envelope_ponderomotive(self._h, ap, op)
        return out

    def envelope_gather(self, problem: int, pond, samples, out=None):
        """|a|^2, A~_rho, A~_z of problem `problem` (its [3, nr, nz] real ponderomotive planes, as
        `ponderomotive` returns them) at the samples (float64 [n, 4] cuda tensor of z, x, y, w): float64
        [n, 3] cuda tensor."""
        import torch
        if not (samples.is_cuda and samples.dtype == torch.float64 and samples.dim() == 2 and samples.shape[1] == 4
                and samples.is_contiguous()):
            raise ValueError("samples: contiguous float64 cuda tensor [n, 4]")
        p = self.problems[problem]
        pp = self._chk(pond, (3, p.nr, p.nz), self._rdtype(), "pond")
        if out is None:
            out = torch.empty((samples.shape[0], 3), dtype=torch.float64, device=samples.device)
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and tuple(out.shape) == (samples.shape[0], 3)):
            raise ValueError("out: contiguous float64 cuda tensor [n, 3]")
        envelope_gather(self._h, problem, pp, samples.data_ptr(), samples.shape[0], out.data_ptr())
        return out

    def query(self) -> dict:
        return fdetd_query(self._h)

    def export_state(self) -> bytes:
        return fdetd_export_state(self._h)

    def import_state(self, blob: bytes):
        fdetd_import_state(self._h, blob)

    def close(self):
        if self._h:
            fdetd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
