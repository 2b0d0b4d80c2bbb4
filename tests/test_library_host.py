"""Host-side checks of the HIP library that need no GPU: it loads, exports every C-ABI symbol declared in
include/fdetd.h, generates its coefficient tables correctly (an independent derivation from the oracle's:
Fornberg's recursion), computes the Taylor stability bound, and rejects bad plans before touching HIP."""
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import paper_2605_12132_amd as F
from paper_2605_12132_amd import binding
from test_oracle_coefficients import exact_axis, exact_d1, exact_d2, exact_halfshift, exact_staggered

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "fdetd.h")).read()
    return sorted(set(re.findall(r"FDETD_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    syms = header_symbols()
    assert len(syms) >= 10, syms
    for s in syms:
        assert hasattr(binding.lib, s), s
    assert sorted(binding.EXPORTS) == syms


@pytest.mark.parametrize("which,fn", [(0, exact_staggered), (1, exact_halfshift), (2, exact_d1), (3, exact_d2),
                                      (4, exact_axis)])
def test_library_coefficients_exact(which, fn):
    for nd in range(1, 17):
        got = np.array(F.fdetd_coefficients(which, nd))
        want = np.array([float(x) for x in fn(nd)])
        assert np.max(np.abs(got - want)) <= 2e-16 * nd * np.max(np.abs(want)) + 1e-300, (which, nd)


def test_taylor_stability_bound():
    # |T_4(ix)|^2 = 1 - x^6/72 + x^8/576 crosses 1 at x = 2 sqrt 2
    assert abs(F.fdetd_taylor_stability_bound(4) - 2 * math.sqrt(2)) < 2e-4
    for N in (8, 12, 16):
        # first positive root of |T_N(ix)|^2 - 1, coefficients in exact rationals (an independent computation)
        re = [Fraction(0)] * (N + 1)
        im = [Fraction(0)] * (N + 1)
        for n in range(N + 1):
            (re if n % 2 == 0 else im)[n] = Fraction((-1) ** (n // 2), math.factorial(n))
        sq = [Fraction(0)] * (2 * N + 1)
        for a in range(N + 1):
            for b in range(N + 1):
                sq[a + b] += re[a] * re[b] + im[a] * im[b]
        sq[0] -= 1
        first = next(k for k, v in enumerate(sq) if v != 0)
        roots = np.polynomial.Polynomial([float(v) for v in sq[first:]]).roots()
        x = min(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 1e-3)
        assert abs(F.fdetd_taylor_stability_bound(N) - x) < 2e-3, (N, x)
    assert abs(F.fdetd_taylor_stability_bound(2) - (8e-9) ** 0.25) < 2e-4  # |T_2(ix)|^2 = 1 + x^4/4
    assert F.fdetd_taylor_stability_bound(9) < 1.0       # N = 1, 2 mod 4: weak growth at every x


@pytest.mark.parametrize("bad", [dict(fd_order=3), dict(fd_order=34), dict(nz=8), dict(nr=8), dict(m=-1),
                                 dict(taylor_order=0), dict(dt=0.0), dict(dz=float("nan"))])
def test_plan_rejects_bad_problems_before_touching_the_gpu(bad):
    p = dict(nz=64, nr=32, m=1, fd_order=16, taylor_order=8, dz=0.3, dr=0.6, dt=0.15)
    p.update(bad)
    with pytest.raises(F.FdetdError) as e:
        F.fdetd_plan([F.Problem(**p)])
    assert e.value.code == binding.FDETD_E_ARG
    assert "problem 0" in F.fdetd_last_error(None)


def test_entry_points_reject_a_null_plan():
    """Every call that takes a plan fails cleanly with FDETD_E_ARG on NULL, before any HIP call."""
    calls = [
        lambda: F.fdetd_gather(None, [0], 0, 0, 0),
        lambda: F.fdetd_gather_supersampled(None, [0], 0, 0, 0, 3),
        lambda: F.fdetd_deposit_rho(None, 0, 0, 0.0, 0.5, [0]),
        lambda: F.fdetd_deposit_current(None, 0, 0, 0.5, [0]),
        lambda: F.envelope_ponderomotive(None, [0], [0]),
        lambda: F.envelope_absorber(None, -1, 4, 4, 1.0, 2.0),
        lambda: F.envelope_gather(None, 0, 0, 0, 0, 0),
    ]
    for call in calls:
        with pytest.raises(F.FdetdError) as e:
            call()
        assert e.value.code == binding.FDETD_E_ARG
        assert "NULL plan" in F.fdetd_last_error(None)


def test_plan_rejects_mixed_kinds_and_bad_flags():
    a = F.Problem(64, 32, 0, 8, 4, 0.3, 0.6, 0.15)
    b = F.Problem(64, 32, 0, 8, 4, 0.3, 0.6, 0.15, kind=F.ENVELOPE)
    with pytest.raises(F.FdetdError):
        F.fdetd_plan([a, b])
    with pytest.raises(F.FdetdError):
        F.fdetd_plan([a], flags=F.PLAN_USE_GRAPH, stream=0)   # graphs need a real stream
    with pytest.raises(F.FdetdError):
        F.fdetd_plan([a], precision=7)
    with pytest.raises(F.FdetdError):
        F.fdetd_plan([a], flags=1024)
    assert "unknown flag" in F.fdetd_last_error(None)
    with pytest.raises(F.FdetdError):  # the increment form is an FP32C Maxwell plan option
        F.fdetd_plan([a], precision=F.FP64, flags=F.PLAN_INCREMENT_FORM)
    assert "FP32C plan" in F.fdetd_last_error(None)


def test_header_layout_matches_binding(tmp_path):
    """The ctypes mirror of the C-ABI agrees with include/fdetd.h as a C compiler reads it: sizes and field
    offsets of both structs, and the value of every constant the binding restates."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"fdetd_problem_desc": binding.ProblemDesc, "fdetd_plan_info": binding.PlanInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fdetd.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    consts = {"FDETD_OK": binding.FDETD_OK, "FDETD_E_ARG": binding.FDETD_E_ARG,
              "FDETD_E_UNSTABLE": binding.FDETD_E_UNSTABLE, "FDETD_E_NOMEM": binding.FDETD_E_NOMEM,
              "FDETD_E_HIP": binding.FDETD_E_HIP, "FDETD_FP64": binding.FP64, "FDETD_FP32C": binding.FP32C,
              "FDETD_MAXWELL": binding.MAXWELL, "FDETD_ENVELOPE": binding.ENVELOPE,
              "FDETD_PLAN_SKIP_STABILITY": binding.PLAN_SKIP_STABILITY, "FDETD_PLAN_USE_GRAPH": binding.PLAN_USE_GRAPH,
              "FDETD_PLAN_PROFILE": binding.PLAN_PROFILE, "FDETD_PLAN_NO_AUTOTUNE": binding.PLAN_NO_AUTOTUNE,
              "FDETD_PLAN_ONE_STREAM": binding.PLAN_ONE_STREAM,
              "FDETD_PLAN_CURRENT_CORRECTION": binding.PLAN_CURRENT_CORRECTION,
              "FDETD_PLAN_MIXED_WIDTHS": binding.PLAN_MIXED_WIDTHS, "FDETD_PLAN_PER_WIDTH": binding.PLAN_PER_WIDTH,
              "FDETD_PLAN_INCREMENT_FORM": binding.PLAN_INCREMENT_FORM,
              "FDETD_PLAN_SEPARATE_WN": binding.PLAN_SEPARATE_WN}
    for k in consts:
        lines.append(f'printf("const {k} %lld\\n", (long long)({k}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for cname, ct in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert got[(cname, f)] == getattr(ct, f).offset, (cname, f)
    for k, v in consts.items():
        assert got[("const", k)] == v, k
