"""Benchmark: field cell-updates/s of the FDETD step on the current-driven workload (modes m = 0, 1 on a
2048 x 256 grid, 16th-order staggered differences, Taylor order 8, dt = dz/2, Gaussian bunch + noise
current, 500 steps), FP64 and FP32-compensated, on one MI355X.

Prints ONE JSON line.  `value` is the FP64 rate (cells x modes x steps / s) over exactly --steps steps,
with every input (fields, the per-step currents of all steps) resident in HBM before the timed region,
replayed from a captured hipGraph.  Also reported:
  roofline     achieved algorithmic HBM bytes / stage-kernel time of the dominant kernel (Maxwell Horner
               stage), from HIP events around every stage launch in a profiled pass of the same workload;
  fp32c        the same measurement for the FP32-compensated path, with its error against the FP64 path;
  cpu_baseline the CPU FP64 oracle timed on a bounded sample (one mode, a few steps) on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "field cell-updates/s (cells×modes×steps/s), FP64 vs FP32-comp at fixed error"
# HBM traffic of the stage kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this benchmark, with the
# hash of the sources the kernel is compiled from and the segment length of the launches counted;
# reported only while both still match (the kernel code, and the tiling the timed plan runs).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_maxwell_stage_current_driven_2048x256_o16_pmc.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2605_12132_amd", "csrc", f)
                  for f in ("fdetd_march.hip", "fdetd_tiles.h", "fdetd_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_currents(w, steps, dtype, seed):
    """Per-step currents [steps, 3, nr, nz] of every problem, generated on the GPU (seeded): the Gaussian
    bunch moving at c on the axis (J_z of mode 0) plus uniform white noise of relative amplitude 1e-3
    (mode 0: real part only) -- the recipe of inputs.bunch_current, drawn with torch's device RNG."""
    import torch
    e = w.extra
    out = []
    g = torch.Generator(device="cuda")
    for p in range(w.n):
        g.manual_seed(seed * 1000 + p)
        nz, nr, m = w.nz[p], w.nr[p], w.m[p]
        rdt = torch.float64
        shape = (steps, 3, nr, nz)
        amp = e["noise"] * e["nb"]
        re = (torch.rand(shape, generator=g, device="cuda", dtype=rdt) * 2 - 1) * amp
        im = torch.zeros_like(re) if m == 0 else (torch.rand(shape, generator=g, device="cuda", dtype=rdt) * 2 - 1) * amp
        if m == 0:
            t = (torch.arange(steps, device="cuda", dtype=rdt) + 0.5) * w.dt
            rp = (torch.arange(nr, device="cuda", dtype=rdt) + 0.5) * w.dr
            zs = (torch.arange(nz, device="cuda", dtype=rdt) - 0.5) * w.dz
            zb = 0.25 * nz * w.dz + t
            bunch = -e["nb"] * torch.exp(-((zs[None, None, :] - zb[:, None, None]) ** 2) / (2 * e["sigz"] ** 2)
                                         - rp[None, :, None] ** 2 / (2 * e["sigr"] ** 2))
            re[:, 2] += bunch
        out.append(torch.complex(re, im).to(dtype).contiguous())
        del re, im
    return out


def energy_weights(w, p):
    """Volume weights w_m r dr dz of the six components (rho-staggered rows at k dr)."""
    rp = (np.arange(w.nr[p]) + 0.5) * w.dr
    rs = np.arange(w.nr[p]) * w.dr
    wm = 2 * math.pi if w.m[p] == 0 else math.pi
    r = np.stack([rs, rp, rp, rp, rs, rs])
    return wm * r * w.dr * w.dz  # [6, nr]


class seg_rows_env:
    """Plans built inside get FDETD_SEG_ROWS = n (no autotuning) when n is given."""

    def __init__(self, n):
        self.n, self.old = n, None

    def __enter__(self):
        if self.n:
            self.old = os.environ.get("FDETD_SEG_ROWS")
            os.environ["FDETD_SEG_ROWS"] = str(self.n)
        return self

    def __exit__(self, *a):
        if self.n:
            if self.old is None:
                del os.environ["FDETD_SEG_ROWS"]
            else:
                os.environ["FDETD_SEG_ROWS"] = self.old
        return False


def run_path(w, precision, steps, warmup, J, use_graph=True, seg_rows=None):
    """Warm up, capture the K-step graph once (untimed, then restore the state), time exactly K steps."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        psi = [torch.zeros((6, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
        flags = F.PLAN_USE_GRAPH if use_graph else 0
        t0 = time.time()
        with seg_rows_env(seg_rows):
            plan = F.Plan(w.problems(), precision=precision, flags=flags)
        plan_s = time.time() - t0
        if warmup:
            plan.step(psi, [j[:warmup] for j in J], n_steps=warmup)
        jt = [j[warmup:warmup + steps] for j in J]
        saved = [x.clone() for x in psi]
        lo = plan.export_state() if precision == F.FP32C else b""
        # capture + one untimed replay of the exact timed call, then restore the state it started from
        plan.step(psi, jt, n_steps=steps)
        for x, s in zip(psi, saved):
            x.copy_(s)
        if precision == F.FP32C:
            stream.synchronize()
            plan.import_state(lo)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        plan.step(psi, jt, n_steps=steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        info = plan.query()
        plan.close()
    return psi, ms, plan_s, info


def profile_pass(w, precision, steps, J, seg_rows):
    """Eager pass with HIP events around every stage kernel: average duration and algorithmic bytes.  The
    plan is given the segment length the timed plan's autotuning picked, so both run the same tiling."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    psi = [torch.zeros((6, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
    with seg_rows_env(seg_rows):
        plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_PROFILE)
    plan.step(psi, [j[:steps] for j in J], n_steps=steps)
    info = plan.query()
    plan.close()
    n = info["profiled_launches"]
    avg_ms = info["profiled_ms"] / n
    bytes_per_launch = info["profiled_bytes"] / n
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic("fp64" if precision == F.FP64 else "fp32c", seg_rows),
                kernel="k_maxwell_stage",
                launches=n, avg_launch_us=round(avg_ms * 1e3, 2), bytes_per_launch=int(bytes_per_launch))


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision_tag, seg_rows):
    """HBM bytes per stage launch (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration) from
    the committed PMC summary, or None when it is missing, was taken on other kernel sources or at
    another segment length than seg_rows."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("traffic_") and ":" in line)
    if fields.get("traffic_source_hash", "").strip() != kernel_source_hash():
        return None
    if fields.get(f"traffic_seg_rows_{precision_tag}", "").strip() != str(seg_rows):
        return None
    v = fields.get(f"traffic_bytes_per_launch_{precision_tag}")
    return int(float(v)) if v else None


def copy_calibration(n_bytes=1 << 30, reps=10):
    """A plain device-to-device copy of n_bytes, reps times: the known-size kernel against which the
    FETCH_SIZE / WRITE_SIZE counters are scaled.  Also times plain streaming kernels (torch elementwise
    ops over the same sizes, read:write ratios 1:1, 2:1, 3:1, 0:1) for the HBM rate a simple stream
    reaches on this GPU."""
    import torch
    n = n_bytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    b, c, d = torch.empty_like(a).uniform_(), torch.empty_like(a).uniform_(), torch.empty_like(a)

    def rate(fn, words):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        return ms, words * n_bytes / (ms * 1e-3) / 1e9

    ms, copy_gbs = rate(lambda: d.copy_(a), 2)
    streams = {"scale_r1w1": rate(lambda: torch.mul(a, 2.0, out=d), 2)[1],
               "add_r2w1": rate(lambda: torch.add(a, b, out=d), 3)[1],
               "addcmul_r3w1": rate(lambda: torch.addcmul(a, b, c, out=d), 4)[1],
               "fill_w1": rate(lambda: d.fill_(1.0), 1)[1]}
    return dict(copy_bytes_read=n_bytes, copy_bytes_written=n_bytes, reps=reps, ms_per_copy=ms, copy_GBs=copy_gbs,
                stream_GBs={k: round(v, 1) for k, v in streams.items()})


def fp32c_errors(w, psi64, psi32):
    num = den = e64 = e32 = 0.0
    ax = []
    for p in range(w.n):
        a = psi64[p].cpu().numpy()
        b = psi32[p].cpu().numpy().astype(np.complex128)
        wt = energy_weights(w, p)[:, :, None]
        num += float(np.sum(wt * np.abs(a - b) ** 2))
        den += float(np.sum(wt * np.abs(a) ** 2))
        e64 += float(np.sum(wt * np.abs(a) ** 2))
        e32 += float(np.sum(wt * np.abs(b) ** 2))
        # on-axis amplitude: E_rho on the axis for m = 1, E_z next to the axis otherwise
        c = 0 if w.m[p] == 1 else 2
        ref = np.max(np.abs(a[c, 0]))
        ax.append(float(np.max(np.abs(a[c, 0] - b[c, 0])) / ref) if ref > 0 else 0.0)
    return dict(field_rel_l2=math.sqrt(num / den), energy_rel_diff=abs(e32 / e64 - 1), axis_amp_rel_err=max(ax))


def cpu_baseline(w, budget_s=12.0):
    """The oracle (plain C, OpenMP over rows) on one mode of the workload with its current, for as many
    steps as fit in the time budget (at least one)."""
    import oracle
    import paper_2605_12132_amd.inputs as I
    p = 1
    g = oracle.Grid(nz=w.nz[p], nr=w.nr[p], m=w.m[p], fd_order=w.fd_order[p], taylor_order=w.taylor_order,
                    dz=w.dz, dr=w.dr, dt=w.dt)
    psi = np.zeros((6, w.nr[p], w.nz[p]), np.complex128)
    J = I.currents(w, p, 8)
    steps, t_total = 0, 0.0
    while steps < 8 and (steps == 0 or t_total + t_total / steps < budget_s):
        t0 = time.time()
        psi = oracle.step(g, psi, J[steps], 1)
        t_total += time.time() - t0
        steps += 1
    cells = w.nz[p] * w.nr[p]
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return dict(value=cells * steps / t_total, unit="cell-updates/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{steps} step(s) of mode m={w.m[p]} ({w.nz[p]}x{w.nr[p]}, order {w.fd_order[p]}, Taylor "
                       f"{w.taylor_order}, with current) in {t_total:.1f} s; host reports {ncpu} usable cores")


def batched_pass(steps, warmup):
    """The batched uneven workload (64 problems, N_z in [512, 4096], N_rho in [64, 512], modes 0..2,
    orders 8..32, Taylor 8, dt = dz/2): FP32C and FP64 plans over all problems, graph replay of `steps`
    steps with a fresh bunch + noise current per step resident in HBM, fields starting at zero.  Reports
    cell-updates/s, the step-level algorithmic HBM rate (plan's bytes per step / step time) and the
    FP32C error against FP64 after the same steps."""
    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I
    w = I.batched_uneven()
    cells = w.cells()
    res, psis = {}, {}
    for tag, prec, cd in (("fp32c", F.FP32C, torch.complex64), ("fp64", F.FP64, torch.complex128)):
        J = make_currents(w, warmup + steps, cd, w.seed)
        torch.cuda.synchronize()
        psi, ms, plan_s, info = run_path(w, prec, steps, warmup, J, True)
        del J
        torch.cuda.empty_cache()
        gbs = info["bytes_per_step"] * steps / (ms * 1e-3) / 1e9
        res[tag] = dict(value=cells * steps / (ms * 1e-3), ms_per_step=ms / steps, algorithmic_GBs=round(gbs, 1),
                        frac=round(gbs / HBM_PEAK_GBS, 4), launches_per_step=info["launches_per_step"],
                        plan_s=round(plan_s, 2), autotune_ms=round(info["autotune_ms"], 1), streams=info["streams"])
        psis[tag] = psi
        log(f"batched {tag}: {ms / steps:.3f} ms/step, {res[tag]['value']:.4g} cell-updates/s, "
            f"{gbs:.0f} GB/s algorithmic ({info['launches_per_step']} launches/step, plan {plan_s:.1f} s)")
    num = den = 0.0
    for a, b in zip(psis["fp64"], psis["fp32c"]):
        d = a - b.to(torch.complex128)
        num += float(torch.sum(torch.abs(d) ** 2))
        den += float(torch.sum(torch.abs(a) ** 2))
    return dict(workload=w.name, problems=w.n, cells=cells, steps=steps, warmup=warmup, graph=True,
                fp32c=res["fp32c"], fp64=res["fp64"], fp32c_vs_fp64=res["fp32c"]["value"] / res["fp64"]["value"],
                fp32c_field_rel_l2=math.sqrt(num / den) if den > 0 else 0.0)


def envelope_pass(steps, layer=32):
    """The envelope-in-plasma workload (4096 x 512, order 8, Taylor 4, dt = dz/2, static chi): FP64 and
    FP32C plans, graph replay of `steps` steps.  Its working set (about 220 MB in FP64) mostly fits the
    256 MB Infinity Cache, so the rate is reported without an HBM fraction.  Each precision is also run
    with absorbing layers (`layer` cells at both z ends and at the outer rho edge, sigma_max half the
    largest the plan's stability bound admits, quadratic grading).  The ponderomotive field of the final
    state (envelope_ponderomotive) is timed apart, and so are those planes at 10^6 samples spread over the
    pulse region (envelope_gather)."""
    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I
    w = I.envelope_plasma()
    a0, at0 = I.envelope_initial(w)
    chi = I.envelope_chi(w)
    cells = w.cells()
    out, res = {}, {}

    def run(prec, cd, rd, absorbing):
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            a = torch.from_numpy(a0).to(device="cuda", dtype=cd)
            at = torch.from_numpy(at0).to(device="cuda", dtype=cd)
            ch = torch.from_numpy(chi).to(device="cuda", dtype=rd)
            plan = F.Plan(w.problems(), precision=prec, flags=F.PLAN_USE_GRAPH)
            smax = 0.0
            if absorbing:
                rho = plan.query()["dt_rho_max"] / w.dt
                smax = 0.5 * (F.fdetd_taylor_stability_bound(w.taylor_order) / (1.02 * w.dt) - rho) / 2
                plan.absorber(layer, layer, smax, 2.0)
            plan.envelope_step([a], [at], [ch], n_steps=steps)      # capture + first replay (untimed)
            a.copy_(torch.from_numpy(a0).to(device="cuda", dtype=cd))
            at.copy_(torch.from_numpy(at0).to(device="cuda", dtype=cd))
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            plan.envelope_step([a], [at], [ch], n_steps=steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            # ponderomotive field of the final state (|a|^2, A~_rho, A~_z), 20 calls
            pond = plan.ponderomotive([a])
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(20):
                plan.ponderomotive([a], pond)
            ev1.record(stream)
            torch.cuda.synchronize()
            pond_us = ev0.elapsed_time(ev1) / 20 * 1e3
            # the same planes at 10^6 samples spread over the pulse (envelope_gather), 5 calls
            n = 10 ** 6
            gs = torch.Generator(device="cuda")
            gs.manual_seed(w.seed)
            smp = torch.rand((n, 4), generator=gs, device="cuda", dtype=torch.float64)
            smp[:, 0] = (0.2 + 0.6 * smp[:, 0]) * w.nz[0] * w.dz
            smp[:, 1] = (smp[:, 1] - 0.5) * w.nr[0] * w.dr
            smp[:, 2] = (smp[:, 2] - 0.5) * w.nr[0] * w.dr
            smp = smp[torch.argsort(smp[:, 0])].contiguous()
            gout = plan.envelope_gather(0, pond[0], smp)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                plan.envelope_gather(0, pond[0], smp, gout)
            ev1.record(stream)
            torch.cuda.synchronize()
            egather_us = ev0.elapsed_time(ev1) / 5 * 1e3
            plan.close()
        return ms, smax, a, at, (pond_us, egather_us)

    for tag, prec, cd, rd in (("fp64", F.FP64, torch.complex128, torch.float64),
                              ("fp32c", F.FP32C, torch.complex64, torch.float32)):
        ms, _, a, at, (pond_us, egather_us) = run(prec, cd, rd, False)
        # ponderomotive algorithmic bytes per cell: the complex envelope read once, three real planes written
        pond_bytes = cells * (2 + 3) * (8 if prec == F.FP64 else 4)
        out[tag] = dict(value=cells * steps / (ms * 1e-3), ms_per_step=ms / steps,
                        ponderomotive_us=round(pond_us, 2), ponderomotive_GBs=round(pond_bytes / (pond_us * 1e3), 1),
                        envelope_gather_1M_samples_us=round(egather_us, 1))
        res[tag] = (a.cpu().numpy().astype(np.complex128), at.cpu().numpy().astype(np.complex128))
        log(f"envelope {tag}: {ms / steps:.4f} ms/step, {out[tag]['value']:.4g} cell-updates/s; ponderomotive "
            f"field {pond_us:.1f} us ({out[tag]['ponderomotive_GBs']:.0f} GB/s algorithmic), at 10^6 samples "
            f"{egather_us:.1f} us")
        ms, smax, _, _, _ = run(prec, cd, rd, True)
        out[tag]["absorbing"] = dict(value=cells * steps / (ms * 1e-3), ms_per_step=ms / steps, lz=layer, lr=layer,
                                     sigma_max=round(smax, 4))
        log(f"envelope {tag} with absorbing layers: {ms / steps:.4f} ms/step")
    x64 = np.concatenate([res["fp64"][0].ravel(), res["fp64"][1].ravel()])
    x32 = np.concatenate([res["fp32c"][0].ravel(), res["fp32c"][1].ravel()])
    return dict(workload=w.name, cells=cells, steps=steps, graph=True, cache_resident=True,
                fp64=out["fp64"], fp32c=out["fp32c"], fp32c_vs_fp64=out["fp32c"]["value"] / out["fp64"]["value"],
                fp32c_rel_l2=float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64)))


def correction_pass(steps, warmup):
    """The current-driven workload with the current correction of section 3.7 every step
    (FDETD_PLAN_CURRENT_CORRECTION): current blocks of J_rho, J_theta, J_z and a planar density
    differential (the bunch + noise recipe for the currents, uniform noise of the same scale for rho_xy),
    graph replay of `steps` steps, FP64 and FP32C, against the same plans without the correction."""
    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I
    w = I.current_driven()
    cells = w.cells()
    out = {}
    for tag, prec, cd in (("fp64", F.FP64, torch.complex128), ("fp32c", F.FP32C, torch.complex64)):
        J = make_currents(w, warmup + steps, cd, w.seed + 7)
        g = torch.Generator(device="cuda")
        g.manual_seed(w.seed + 8)
        J4 = []
        for j in J:
            rxy = (torch.rand(j[:, :1].shape, generator=g, device="cuda", dtype=torch.float64) * 2 - 1)
            rxy = (rxy * w.extra["noise"] * w.extra["nb"]).to(cd)
            J4.append(torch.cat([j, rxy], dim=1).contiguous())
            del rxy
        res = {}
        for corr in (False, True):
            stream = torch.cuda.Stream()
            stream.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(stream):
                psi = [torch.zeros((6, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
                flags = F.PLAN_USE_GRAPH | (F.PLAN_CURRENT_CORRECTION if corr else 0)
                plan = F.Plan(w.problems(), precision=prec, flags=flags)
                cur = J4 if corr else J
                plan.step(psi, [j[:warmup] for j in cur], n_steps=warmup)
                jt = [j[warmup:warmup + steps] for j in cur]
                plan.step(psi, jt, n_steps=steps)  # capture + first replay (untimed)
                torch.cuda.synchronize()
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                plan.step(psi, jt, n_steps=steps)
                ev1.record(stream)
                torch.cuda.synchronize()
                ms = ev0.elapsed_time(ev1)
                plan.close()
            res[corr] = ms / steps
        del J, J4
        torch.cuda.empty_cache()
        out[tag] = dict(value=cells * steps / (res[True] * steps * 1e-3), ms_per_step=res[True],
                        ms_per_step_without=res[False], overhead=res[True] / res[False] - 1.0)
        log(f"correction {tag}: {res[True]:.4f} ms/step with, {res[False]:.4f} without")
    return dict(workload=w.name + "_corrected", cells=cells, steps=steps, graph=True, fp64=out["fp64"],
                fp32c=out["fp32c"])


def lwfa_pass(steps, warmup, n_samples=10 ** 6):
    """The LWFA-scale workload (modes 0, 1, 2 on 8192 x 1024, order 32, Taylor 8, dt = dz/2): the current of
    each step is a bunch of n_samples point samples (Gaussian, sigma_z = 2 um, sigma_rho = 1 um, total charge
    of peak density n_b) moving at c, in z order, deposited with fdetd_deposit_jz (timed separately,
    including the advance of the sample positions; all currents and rho_xy of the same samples with a
    transverse velocity spread, fdetd_deposit_current, and their charge density, fdetd_deposit_rho, timed
    apart), then graph replay of `steps` field
    steps, then the fields of the final state at the samples (fdetd_gather, timed apart, also with 2x
    supersampling along z and rho).  FP64 and FP32C; the FP32C error against FP64 after the same steps."""
    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I
    w = I.lwfa_scale()
    e = w.extra
    nz, nr = w.nz[0], w.nr[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed)
    base = torch.randn((n_samples, 4), generator=g, device="cuda", dtype=torch.float64)
    base[:, 0] = 0.25 * nz * w.dz + e["sigz"] * base[:, 0]
    base[:, 1:3] *= e["sigr"]
    base[:, 3] = -e["nb"] * (2 * math.pi) ** 1.5 * e["sigz"] * e["sigr"] ** 2 / n_samples
    # position order, as a PIC code keeps its particles (all samples move alike, so it holds every step):
    # blocks of consecutive samples then deposit through LDS tiles
    base = base[torch.argsort(base[:, 0])].contiguous()
    cells = w.cells()
    res, psis = {}, {}
    for tag, prec, cd in (("fp64", F.FP64, torch.complex128), ("fp32c", F.FP32C, torch.complex64)):
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            plan = F.Plan(w.problems(), precision=prec, flags=0)
            J = [torch.zeros((warmup + steps, 3, nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            smp = base.clone()
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for st in range(warmup + steps):
                smp[:, 0] = base[:, 0] + (st + 0.5) * w.dt
                plan.deposit_jz(smp, [j[st] for j in J], vz=1.0, eps=0.5)
            ev1.record(stream)
            torch.cuda.synchronize()
            dep_ms = ev0.elapsed_time(ev1) / (warmup + steps)
            plan.close()
            # all currents of moving samples (J_rho, J_theta, modified-Esirkepov J_z and rho_xy of the
            # current correction): the bunch with a transverse velocity spread, 5 calls
            plan = F.Plan(w.problems(), precision=prec,
                          flags=F.PLAN_CURRENT_CORRECTION | F.PLAN_SKIP_STABILITY | F.PLAN_NO_AUTOTUNE)
            J4 = [torch.zeros((4, nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            s8 = torch.zeros((n_samples, 8), dtype=torch.float64, device="cuda")
            s8[:, :4] = smp
            s8[:, 4:6] = 0.01 * torch.randn((n_samples, 2), generator=g, device="cuda", dtype=torch.float64)
            s8[:, 6] = 0.999
            plan.deposit_current(s8, J4)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                plan.deposit_current(s8, J4)
            ev1.record(stream)
            torch.cuda.synchronize()
            dep_cur_ms = ev0.elapsed_time(ev1) / 5
            # charge density of the same samples (fdetd_deposit_rho), 5 calls
            R1 = [torch.zeros((nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            plan.deposit_rho(smp, R1)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                plan.deposit_rho(smp, R1)
            ev1.record(stream)
            torch.cuda.synchronize()
            dep_rho_ms = ev0.elapsed_time(ev1) / 5
            plan.close()
            del J4, s8, R1
        psi, ms, plan_s, info = run_path(w, prec, steps, warmup, J, True)
        del J
        torch.cuda.empty_cache()
        # fields of the final state at the samples' last positions (destaggering + interpolation), 5 calls
        with torch.cuda.stream(stream):
            plan = F.Plan(w.problems(), precision=prec, flags=F.PLAN_SKIP_STABILITY | F.PLAN_NO_AUTOTUNE)
            fields = plan.gather(psi, smp)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                plan.gather(psi, smp, fields)
            ev1.record(stream)
            torch.cuda.synchronize()
            gather_ms = ev0.elapsed_time(ev1) / 5
            # the same with 2x supersampling along z and rho (fdetd_gather_supersampled)
            plan.gather(psi, smp, fields, supersample=3)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(5):
                plan.gather(psi, smp, fields, supersample=3)
            ev1.record(stream)
            torch.cuda.synchronize()
            gather_ss_ms = ev0.elapsed_time(ev1) / 5
            plan.close()
        gbs = info["bytes_per_step"] * steps / (ms * 1e-3) / 1e9
        res[tag] = dict(value=cells * steps / (ms * 1e-3), ms_per_step=ms / steps, algorithmic_GBs=round(gbs, 1),
                        frac=round(gbs / HBM_PEAK_GBS, 4), deposit_ms_per_step=dep_ms, gather_ms=gather_ms,
                        gather_supersampled_ms=gather_ss_ms, deposit_current_ms=dep_cur_ms,
                        deposit_rho_ms=dep_rho_ms,
                        seg_rows=info["seg_rows"])
        psis[tag] = psi
        log(f"lwfa {tag}: {ms / steps:.3f} ms/step, {res[tag]['value']:.4g} cell-updates/s, {gbs:.0f} GB/s "
            f"algorithmic; deposition of {n_samples} samples {dep_ms:.3f} ms/step (all currents and rho_xy "
            f"{dep_cur_ms:.3f} ms, charge density {dep_rho_ms:.3f} ms); gather {gather_ms:.3f} ms, "
            f"2x supersampled (z and rho) {gather_ss_ms:.3f} ms")
    num = den = 0.0
    for a, b in zip(psis["fp64"], psis["fp32c"]):
        num += float(torch.sum(torch.abs(a - b.to(torch.complex128)) ** 2))
        den += float(torch.sum(torch.abs(a) ** 2))
    return dict(workload=w.name, cells=cells, steps=steps, warmup=warmup, samples=n_samples, graph=True,
                fp64=res["fp64"], fp32c=res["fp32c"], fp32c_vs_fp64=res["fp32c"]["value"] / res["fp64"]["value"],
                fp32c_field_rel_l2=math.sqrt(num / den) if den > 0 else 0.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--seg-rows-fp64", type=int, default=None,
                    help="fixed rows per marching segment of the FP64 plans instead of plan-time autotuning")
    ap.add_argument("--seg-rows-fp32c", type=int, default=None, help="the same for the FP32C plans")
    ap.add_argument("--batched-steps", type=int, default=20,
                    help="steps of the 64-problem batched workload reported beside the headline (0: skip)")
    ap.add_argument("--lwfa-steps", type=int, default=20,
                    help="steps of the LWFA-scale workload reported beside the headline (0: skip)")
    ap.add_argument("--correction-steps", type=int, default=50,
                    help="steps of the current-driven workload with the current correction (0: skip)")
    ap.add_argument("--envelope-steps", type=int, default=2000,
                    help="steps of the envelope workload reported beside the headline (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain 1 GiB device copy used to scale the rocprofv3 byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the problems of this workload are "
              "independent modes and would be distributed one plan per GPU with no communication.", flush=True)
        sys.exit(2)

    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I

    if args.calibrate_copy:
        print(json.dumps(copy_calibration()), flush=True)
        return
    w = I.current_driven()
    K, W = args.steps, args.warmup
    cells = w.cells()
    log(f"workload {w.name}: {w.n} modes x {w.nz[0]}x{w.nr[0]}, order {w.fd_order[0]}, N={w.taylor_order}, "
        f"K={K}, W={W}")
    t0 = time.time()
    J64 = make_currents(w, W + K, torch.complex128, w.seed)
    torch.cuda.synchronize()
    log(f"currents resident: {sum(j.numel() for j in J64) * 16 / 1e9:.1f} GB in {time.time() - t0:.1f} s")

    psi64, ms64, plan_s, info64 = run_path(w, F.FP64, K, W, J64, not args.no_graph, args.seg_rows_fp64)
    rate64 = cells * K / (ms64 * 1e-3)
    log(f"FP64: {ms64 / K:.4f} ms/step, {rate64:.4g} cell-updates/s (plan {plan_s:.2f} s, dt*rho {info64['dt_rho_max']:.3f})")
    prof_steps = min(args.profile_steps, K + W)  # the currents held resident cover K + W steps
    roof64 = profile_pass(w, F.FP64, prof_steps, J64, info64["seg_rows"])
    log(f"FP64 stage kernel: {roof64['avg_launch_us']} us/launch, {roof64['achieved']} GB/s ({roof64['frac'] * 100:.1f}% of HBM)")

    fp32c = None
    if not args.fp64_only:
        J32 = [j.to(torch.complex64) for j in J64]
        del J64
        torch.cuda.empty_cache()
        psi32, ms32, _, info32 = run_path(w, F.FP32C, K, W, J32, not args.no_graph, args.seg_rows_fp32c)
        rate32 = cells * K / (ms32 * 1e-3)
        roof32 = profile_pass(w, F.FP32C, prof_steps, J32, info32["seg_rows"])
        errs = fp32c_errors(w, psi64, psi32)
        log(f"FP32C: {ms32 / K:.4f} ms/step, {rate32:.4g} cell-updates/s, errors {errs}")
        fp32c = dict(value=rate32, ms_per_step=ms32 / K, dtype="f32+comp", vs_fp64=rate32 / rate64, roofline=roof32,
                     error_vs_fp64_after_steps=W + K, **errs,
                     tiling=dict(seg_rows=info32["seg_rows"], seg_rows_axis=info32["seg_rows_axis"],
                                 autotune_ms=round(info32["autotune_ms"], 1)))
        del J32
    else:
        del J64

    batched = None
    if args.batched_steps > 0 and not args.fp64_only:
        del psi64
        torch.cuda.empty_cache()
        batched = batched_pass(args.batched_steps, W)
    envelope = envelope_pass(args.envelope_steps) if args.envelope_steps > 0 and not args.fp64_only else None
    lwfa = lwfa_pass(args.lwfa_steps, W) if args.lwfa_steps > 0 and not args.fp64_only else None
    correction = (correction_pass(args.correction_steps, W)
                  if args.correction_steps > 0 and not args.fp64_only else None)
    cpu = None if args.no_cpu else cpu_baseline(w)
    if cpu:
        log(f"CPU oracle: {cpu['value']:.4g} cell-updates/s on {cpu['cores']} threads ({cpu['sample']})")
    out = {
        "metric": METRIC, "value": rate64, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms64 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "modes": w.m, "nz": w.nz[0], "nr": w.nr[0], "fd_order": w.fd_order[0],
                   "taylor_order": w.taylor_order, "dt_over_dz": 0.5, "dr_over_dz": 2.0, "current": "bunch+noise",
                   "graph": not args.no_graph, "parallelism": "single GPU, modes batched in one plan"},
        "roofline": roof64,
        "cpu_baseline": cpu,
        "tiling": dict(seg_rows=info64["seg_rows"], autotune_ms=round(info64["autotune_ms"], 1)),
        "fp32c": fp32c,
        "batched": batched,
        "envelope": envelope,
        "lwfa": lwfa,
        "correction": correction,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
