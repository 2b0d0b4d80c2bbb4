"""Benchmark: field cell-updates/s of the FDETD step on the LWFA-scale workload -- modes m = 0, 1, 2 on an
8192 x 1024 grid, 32nd-order staggered differences, Taylor order 8, dt = dz/2, the current of 10^6 bunch
samples moving at c deposited every step -- the largest single-GPU workload, FP64 and FP32-compensated, on
one MI355X.

Prints ONE JSON line.  A step is one pass of the whole hot path: the step's current (J_z of every mode
deposited from the samples at the step's midpoint positions), current staging, the Horner stages with the
midpoint source and the axis rule.  `value` is the FP64 rate (cells x modes x steps / s) over exactly
--steps steps of fdetd_step_graph, the K-step loop captured as one hipGraph and replayed, with the fields
and the samples resident in HBM when timing starts.  Also reported:
  roofline      the dominant kernel (the Maxwell Horner stage): algorithmic HBM bytes per launch (21
                complex values per cell, 336 B FP64 / 168 B FP32) over its average duration, from HIP
                events around every stage launch of a profiled pass (the plan's stream), with the HBM
                traffic of the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary;
  fp32c         the same for the FP32-compensated path, with its error against the FP64 path;
  full_length   both precisions over the workload's 1000 steps, and the FP32C error after them;
  cpu_baseline  the CPU FP64 oracle timed on a bounded sample on the host cores (all cores and one);
  current_driven, batched, envelope, correction, sources: the other workloads and the source kernels.
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
# HBM traffic of the stage kernel on the LWFA-scale workload from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# with the hash of the sources the kernel is compiled from and the segment length of the launches
# counted; reported only while both still match (the kernel code, and the tiling the timed plan runs).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_maxwell_stage_lwfa_m012_8192x1024_o32_pmc.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2605_12132_amd", "csrc", f)
                  for f in ("fdetd_march.hip", "fdetd_tiles.h", "fdetd_internal.h")]
N_SAMPLES = 10 ** 6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_stage(precision):
    """Algorithmic HBM bytes of one Horner stage per cell with a current: read v (6c), psi (6c), Jbar (3c),
    write v (6c)."""
    import paper_2605_12132_amd as F
    return 21 * (16 if precision == F.FP64 else 8)


def energy_weights(w, p):
    """Volume weights w_m r dr dz of the six components (rho-staggered rows at k dr), [6, nr, 1]."""
    import torch
    rp = (torch.arange(w.nr[p], dtype=torch.float64, device="cuda") + 0.5) * w.dr
    rs = torch.arange(w.nr[p], dtype=torch.float64, device="cuda") * w.dr
    wm = 2 * math.pi if w.m[p] == 0 else math.pi
    return (wm * torch.stack([rs, rp, rp, rp, rs, rs]) * w.dr * w.dz)[:, :, None]


def fp32c_errors(w, psi64, psi32):
    """Energy-weighted field rel. L2 of FP32C against FP64, relative energy difference, and the on-axis
    amplitude error (E_rho on the axis for m = 1, E_z next to it otherwise), computed on the GPU."""
    import torch
    num = den = e32 = 0.0
    ax = []
    for p in range(w.n):
        a, b = psi64[p], psi32[p].to(torch.complex128)
        wt = energy_weights(w, p)
        num += float(torch.sum(wt * torch.abs(a - b) ** 2))
        den += float(torch.sum(wt * torch.abs(a) ** 2))
        e32 += float(torch.sum(wt * torch.abs(b) ** 2))
        c = 0 if w.m[p] == 1 else 2
        ref = float(torch.max(torch.abs(a[c, 0])))
        ax.append(float(torch.max(torch.abs(a[c, 0] - b[c, 0]))) / ref if ref > 0 else 0.0)
    return dict(field_rel_l2=math.sqrt(num / den) if den > 0 else 0.0,
                energy_rel_diff=abs(e32 / den - 1) if den > 0 else 0.0, axis_amp_rel_err=max(ax))


def lwfa_samples(w, n=N_SAMPLES):
    """The bunch of the LWFA-scale workload as n point samples at t = 0 (Gaussian, sigma_z = 2 um,
    sigma_rho = 1 um, total charge of peak density n_b, centred at a quarter of the box), in z order as a
    PIC code keeps its particles.  Seeded, drawn on the GPU."""
    import torch
    e = w.extra
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed)
    s = torch.randn((n, 4), generator=g, device="cuda", dtype=torch.float64)
    s[:, 0] = 0.25 * w.nz[0] * w.dz + e["sigz"] * s[:, 0]
    s[:, 1:3] *= e["sigr"]
    s[:, 3] = -e["nb"] * (2 * math.pi) ** 1.5 * e["sigz"] * e["sigr"] ** 2 / n
    return s[torch.argsort(s[:, 0])].contiguous()


def sample_jgen(smp, step0):
    import paper_2605_12132_amd as F
    return F.Jgen(F.JGEN_SAMPLES, step0=step0, samples=smp, vz=1.0, eps=0.5)


def bunch_jgen(w, step0):
    """The bunch + noise current recipe of the current-driven and batched workloads, made in the graph."""
    import paper_2605_12132_amd as F
    e = w.extra
    return F.Jgen(F.JGEN_BUNCH, step0=step0, seed=w.seed, nb=e["nb"], sigz=e["sigz"], sigr=e["sigr"], z0_frac=0.25,
                  vb=1.0, noise=e["noise"])


class seg_rows_env:
    """Plans built inside get FDETD_SEG_ROWS = n (no autotuning) when n is given, the store policy of the
    stage outputs FDETD_STORE_POLICY = store_policy (0 default, 1 non-temporal) and the tile numbering
    FDETD_TILE_ORDER = tile_order (0 half first, 1 segment first) when those are given."""

    def __init__(self, n, store_policy=None, tile_order=None):
        self.set = {}
        if n:
            self.set["FDETD_SEG_ROWS"] = str(n)
        if store_policy is not None:
            self.set["FDETD_STORE_POLICY"] = str(int(store_policy))
        if tile_order is not None:
            self.set["FDETD_TILE_ORDER"] = str(int(tile_order))
        self.old = {}

    def __enter__(self):
        for k, v in self.set.items():
            self.old[k] = os.environ.get(k)
            os.environ[k] = v
        return self

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
        return False


def initial_state(w, cd):
    """Initial fields of every problem on the GPU (the workload's Gaussian pulse, or zeros)."""
    import torch
    import paper_2605_12132_amd.inputs as I
    return [torch.from_numpy(I.initial_fields(w, p)).to(device="cuda", dtype=cd) for p in range(w.n)]


def run_graph_path(w, precision, steps, warmup, jgen_of, seg_rows=None, use_graph=True, extra_flags=0,
                   store_policy=None, tile_order=None):
    """Warm up W steps, capture the K-step loop of fdetd_step_graph once (untimed, then restore the state),
    time exactly K steps of its replay.  jgen_of(step0) gives the step generator of the call."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        psi = initial_state(w, cd)
        jw = [torch.zeros((3, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
        flags = (F.PLAN_USE_GRAPH if use_graph else 0) | extra_flags
        t0 = time.time()
        with seg_rows_env(seg_rows, store_policy, tile_order):
            plan = F.Plan(w.problems(), precision=precision, flags=flags)
        plan_s = time.time() - t0
        if warmup:
            plan.step_graph(psi, jgen_of(0), jw, n_steps=warmup)
        saved = [x.clone() for x in psi]
        lo = plan.export_state() if precision == F.FP32C else b""
        t0 = time.time()
        plan.step_graph(psi, jgen_of(warmup), jw, n_steps=steps)  # capture + first replay (untimed)
        torch.cuda.synchronize()
        capture_s = time.time() - t0
        for x, s in zip(psi, saved):
            x.copy_(s)
        del saved
        if precision == F.FP32C:
            stream.synchronize()
            plan.import_state(lo)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        plan.step_graph(psi, jgen_of(warmup), jw, n_steps=steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        info = plan.query()
        plan.close()
    del jw
    return psi, ms, dict(plan_s=round(plan_s, 2), capture_and_first_replay_s=round(capture_s, 2)), info


def profile_pass(w, precision, steps, jgen_of, seg_rows, seg_axis=0, store_policy=None, tile_order=None):
    """Eager pass with HIP events around every stage kernel on the plan's stream: average duration and
    algorithmic bytes (21 complex values per cell).  The plan is given the segment length the timed plan's
    autotuning picked, so both run the same tiling."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    psi = initial_state(w, cd)
    jw = [torch.zeros((3, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
    with seg_rows_env(seg_rows, store_policy, tile_order):
        plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_PROFILE)
    plan.step_graph(psi, jgen_of(0), jw, n_steps=steps)
    info = plan.query()
    plan.close()
    n = info["profiled_launches"]
    avg_ms = info["profiled_ms"] / n
    bytes_per_launch = w.cells() * bytes_per_stage(precision)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic("fp64" if precision == F.FP64 else "fp32c", seg_rows, seg_axis,
                                         info["store_policy"], info["tile_order"]),
                kernel="k_maxwell_stage", launches=n, avg_launch_us=round(avg_ms * 1e3, 2),
                bytes_per_launch=int(bytes_per_launch), bytes_per_cell=bytes_per_stage(precision),
                timing="HIP events around each stage launch on the plan's stream, eager pass of "
                       f"{steps} steps (every stage counted at 21 complex values per cell)")


def kernel_source_hash():
    """Hash of the stage kernel's sources without their comments (the text from // to the end of a line)
    and blank lines, so that an edit of a comment keeps the counters taken on the same code."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(precision_tag, seg_rows, seg_axis=0, store_policy=0, tile_order=0):
    """HBM bytes per stage launch (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration) from
    the committed PMC summary, or None when it is missing, was taken on other kernel sources, holds no
    figure for this tiling (segments of seg_rows rows, store policy of the stage outputs, tile order), or
    (FP32C) was taken with other near-axis segments."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("traffic_") and ":" in line)
    if fields.get("traffic_source_hash", "").strip() != kernel_source_hash():
        return None
    if seg_axis and fields.get("traffic_seg_axis_fp32c", "").strip() != str(seg_axis):
        return None
    v = fields.get(f"traffic_bytes_per_launch_{precision_tag}_seg{seg_rows}_pol{int(store_policy)}_ord{int(tile_order)}")
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


def graph_workload_pass(w, steps, warmup, tag, extra_flags=0):
    """A workload with the bunch + noise current made in the graph (fdetd_step_graph, FDETD_JGEN_BUNCH):
    FP64 and FP32C, K steps timed as above; cell-updates/s, the step-level algorithmic HBM rate (the plan's
    bytes per step / step time), launches per step and the FP32C error against FP64."""
    import paper_2605_12132_amd as F
    cells = w.cells()
    res, psis = {}, {}
    for pt, prec in (("fp64", F.FP64), ("fp32c", F.FP32C)):
        psi, ms, times, info = run_graph_path(w, prec, steps, warmup, lambda s0: bunch_jgen(w, s0),
                                              extra_flags=extra_flags)
        gbs = info["bytes_per_step"] * steps / (ms * 1e-3) / 1e9
        res[pt] = dict(value=cells * steps / (ms * 1e-3), ms_per_step=ms / steps, algorithmic_GBs=round(gbs, 1),
                       frac=round(gbs / HBM_PEAK_GBS, 4), launches_per_step=info["launches_per_step"],
                       streams=info["streams"], autotune_ms=round(info["autotune_ms"], 1), **times)
        psis[pt] = psi
        log(f"{tag} {pt}: {ms / steps:.3f} ms/step, {res[pt]['value']:.4g} cell-updates/s, {gbs:.0f} GB/s "
            f"algorithmic ({info['launches_per_step']} launches/step, plan {times['plan_s']} s, capture + first "
            f"replay {times['capture_and_first_replay_s']} s)")
    errs = fp32c_errors(w, psis["fp64"], psis["fp32c"])
    return dict(workload=w.name, problems=w.n, cells=cells, steps=steps, warmup=warmup, graph=True,
                current="bunch + SplitMix64 noise made in the graph", fp64=res["fp64"], fp32c=res["fp32c"],
                fp32c_vs_fp64=res["fp32c"]["value"] / res["fp64"]["value"], fp32c_error_vs_fp64=errs)


def batched_profile(w, precision, steps, extra_flags=0):
    """Eager pass of the batched workload with HIP events around every stage launch (one stream): the
    stage kernels' aggregate rate at 21 complex values per cell and stage, and the launches per step."""
    import torch
    import paper_2605_12132_amd as F
    cd = torch.complex128 if precision == F.FP64 else torch.complex64
    psi = initial_state(w, cd)
    jw = [torch.zeros((3, w.nr[p], w.nz[p]), dtype=cd, device="cuda") for p in range(w.n)]
    plan = F.Plan(w.problems(), precision=precision, flags=F.PLAN_PROFILE | extra_flags)
    plan.step_graph(psi, bunch_jgen(w, 0), jw, n_steps=steps)
    info = plan.query()
    plan.close()
    n, ms = info["profiled_launches"], info["profiled_ms"]
    bytes_total = steps * w.taylor_order * w.cells() * bytes_per_stage(precision)
    achieved = bytes_total / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None, kernel="k_maxwell_stage",
                launches=n, avg_launch_us=round(ms / n * 1e3, 2), stage_ms_per_step=round(ms / steps, 4),
                bytes_per_step=int(bytes_total / steps), bytes_per_cell=bytes_per_stage(precision),
                timing=f"HIP events around each stage launch, eager pass of {steps} steps on one stream "
                       "(every stage counted at 21 complex values per cell)")


def batched_main(args):
    """--workload batched: the 64-problem uneven batch alone (graph path, default launch grouping), with the
    stage kernels' aggregate rate from an eager pass; for profiling its launches apart from the headline."""
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I
    w = I.batched_uneven()
    K, W = args.steps, args.warmup
    extra = F.PLAN_PER_WIDTH if args.grouping == "per-width" else (F.PLAN_MIXED_WIDTHS if args.grouping == "mixed" else 0)
    res = graph_workload_pass(w, K, W, f"batched ({args.grouping} grouping)", extra)
    roof = {pt: batched_profile(w, prec, args.profile_steps, extra) for pt, prec in (("fp64", F.FP64), ("fp32c", F.FP32C))}
    for pt in roof:
        log(f"batched {pt} stage kernels: {roof[pt]['stage_ms_per_step']} ms per step, {roof[pt]['achieved']} GB/s "
            f"({roof[pt]['frac'] * 100:.1f}% of HBM), {roof[pt]['launches'] // args.profile_steps} stage launches per step")
    r64, r32 = res["fp64"], res["fp32c"]
    out = {
        "metric": METRIC, "value": r64["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": r64["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "problems": w.n, "cells": w.cells(), "taylor_order": w.taylor_order,
                   "fd_orders": sorted(set(w.fd_order)), "grouping": args.grouping, "graph": True,
                   "current": "bunch + SplitMix64 noise made in the graph", "parallelism": "single GPU"},
        "roofline": roof["fp64"], "cpu_baseline": None, "launches_per_step": r64["launches_per_step"],
        "fp32c": dict(r32, roofline=roof["fp32c"], dtype="f32+comp"),
        "fp32c_error_vs_fp64": res["fp32c_error_vs_fp64"],
    }
    print(json.dumps(out), flush=True)


def sources_pass(w, smp):
    """Source and interpolation kernels on the LWFA-scale grid and the 10^6 z-ordered samples, timed apart:
    J_z deposition (fdetd_deposit_jz), all currents and rho_xy of the samples with a transverse velocity
    spread (fdetd_deposit_current), their charge density (fdetd_deposit_rho), and the fields at the samples
    (fdetd_gather, and with 2x supersampling along z and rho)."""
    import torch
    import paper_2605_12132_amd as F
    nz, nr = w.nz[0], w.nr[0]
    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(stream, fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed + 1)
    for tag, prec, cd in (("fp64", F.FP64, torch.complex128), ("fp32c", F.FP32C, torch.complex64)):
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            plan = F.Plan(w.problems(), precision=prec, flags=F.PLAN_SKIP_STABILITY | F.PLAN_NO_AUTOTUNE)
            J = [torch.zeros((3, nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            dep = timed(stream, lambda: plan.deposit_jz(smp, J, vz=1.0, eps=0.5))
            R1 = [torch.zeros((nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            rho = timed(stream, lambda: plan.deposit_rho(smp, R1))
            psi = initial_state(w, cd)
            fields = plan.gather(psi, smp)
            gat = timed(stream, lambda: plan.gather(psi, smp, fields))
            gss = timed(stream, lambda: plan.gather(psi, smp, fields, supersample=3))
            plan.close()
            del J, R1, psi, fields
            torch.cuda.empty_cache()
            plan = F.Plan(w.problems(), precision=prec,
                          flags=F.PLAN_CURRENT_CORRECTION | F.PLAN_SKIP_STABILITY | F.PLAN_NO_AUTOTUNE)
            J4 = [torch.zeros((4, nr, nz), dtype=cd, device="cuda") for _ in range(w.n)]
            s8 = torch.zeros((smp.shape[0], 8), dtype=torch.float64, device="cuda")
            s8[:, :4] = smp
            s8[:, 4:6] = 0.01 * torch.randn((smp.shape[0], 2), generator=g, device="cuda", dtype=torch.float64)
            s8[:, 6] = 0.999
            cur = timed(stream, lambda: plan.deposit_current(s8, J4))
            plan.close()
            del J4, s8
            torch.cuda.empty_cache()
        out[tag] = dict(deposit_jz_ms=round(dep, 4), deposit_rho_ms=round(rho, 4), deposit_current_ms=round(cur, 4),
                        gather_ms=round(gat, 4), gather_supersampled_ms=round(gss, 4))
        log(f"sources {tag}: deposit_jz {dep:.3f} ms, deposit_rho {rho:.3f} ms, deposit_current {cur:.3f} ms, "
            f"gather {gat:.3f} ms, supersampled {gss:.3f} ms")
    return dict(workload=w.name, samples=int(smp.shape[0]), **out)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w):
    """The oracle (plain C, FP64, OpenMP over rows), as it stands: one step of mode m = 1 of the workload
    with a current of the workload's shape (the bunch + noise recipe of inputs.graph_bunch_current), on all
    host cores, and one step of the same mode on a 1024-column window on one core.  Deposition is not
    timed (it is not part of the field step)."""
    import oracle
    import paper_2605_12132_amd.inputs as I
    p = 1
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()

    def rate(nz, threads):
        oracle.set_num_threads(threads)
        wl = w.shrink(nz=nz)
        g = oracle.Grid(nz=nz, nr=w.nr[p], m=w.m[p], fd_order=w.fd_order[p], taylor_order=w.taylor_order,
                        dz=w.dz, dr=w.dr, dt=w.dt)
        psi = np.zeros((6, w.nr[p], nz), np.complex128)
        wl.extra = dict(w.extra, noise=1e-3)
        J = I.graph_bunch_current(wl, p, 0, w.seed)
        t0 = time.time()
        oracle.step(g, psi, J, 1)
        dt = time.time() - t0
        return nz * w.nr[p] / dt, dt, oracle.num_threads()

    v_all, t_all, c_all = rate(w.nz[p], ncpu)
    v_one, t_one, _ = rate(1024, 1)
    oracle.set_num_threads(ncpu)
    return dict(value=v_all, unit="cell-updates/s", cores=c_all, kind="oracle",
                sample=f"1 step of mode m={w.m[p]} ({w.nz[p]}x{w.nr[p]}, order {w.fd_order[p]}, Taylor "
                       f"{w.taylor_order}, with current) in {t_all:.1f} s on {c_all} threads",
                one_core=dict(value=v_one, cores=1,
                              sample=f"1 step of mode m={w.m[p]} on a 1024x{w.nr[p]} window in {t_one:.1f} s"),
                cpu_model=cpu_model(), host_cores=ncpu)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps K of the headline")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--headline-only", action="store_true", help="only the headline FP64 / FP32C lines and roofline")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--seg-rows-fp64", type=int, default=None,
                    help="fixed rows per marching segment of the FP64 plans instead of plan-time autotuning")
    ap.add_argument("--seg-rows-fp32c", type=int, default=None, help="the same for the FP32C plans")
    ap.add_argument("--full-steps", type=int, default=1000,
                    help="steps of the full-length LWFA-scale run reported beside the headline (0: skip)")
    ap.add_argument("--current-driven-steps", type=int, default=500, help="0: skip")
    ap.add_argument("--batched-steps", type=int, default=200, help="0: skip")
    ap.add_argument("--correction-steps", type=int, default=50, help="0: skip")
    ap.add_argument("--envelope-steps", type=int, default=2000, help="0: skip")
    ap.add_argument("--workload", choices=("lwfa", "batched", "envelope"), default="lwfa",
                    help="lwfa: the headline (LWFA-scale grid); batched: the 64-problem uneven batch alone; "
                         "envelope: the envelope-in-plasma workload alone")
    ap.add_argument("--grouping", choices=("default", "per-width", "mixed"), default="default",
                    help="launch grouping of the batched workload's stencil widths")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain 1 GiB device copy used to scale the rocprofv3 byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build measures one GPU's share. "
              "The modes and batched problems are independent and would be distributed one plan per GPU; a grid "
              "too large for one GPU would be split into z-slabs with an N_D-column halo per stage.", flush=True)
        sys.exit(2)

    import torch
    import paper_2605_12132_amd as F
    import paper_2605_12132_amd.inputs as I

    if args.calibrate_copy:
        print(json.dumps(copy_calibration()), flush=True)
        return
    if args.workload == "batched":
        batched_main(args)
        return
    if args.workload == "envelope":
        env = envelope_pass(args.envelope_steps)
        print(json.dumps({"metric": METRIC, "value": env["fp64"]["value"], "unit": "cell-updates/s", "n_gpus": 1,
                          "steps": args.envelope_steps, "ms_per_step": env["fp64"]["ms_per_step"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": env["workload"]}, "roofline": None,
                          "cpu_baseline": None, "envelope": env}), flush=True)
        return
    w = I.lwfa_scale()
    K, W = args.steps, args.warmup
    cells = w.cells()
    log(f"workload {w.name}: {w.n} modes x {w.nz[0]}x{w.nr[0]}, order {w.fd_order[0]}, N={w.taylor_order}, "
        f"{N_SAMPLES} samples deposited per step, K={K}, W={W}")
    smp = lwfa_samples(w)
    jg = lambda s0: sample_jgen(smp, s0)  # noqa: E731

    psi64, ms64, t64, info64 = run_graph_path(w, F.FP64, K, W, jg, args.seg_rows_fp64)
    rate64 = cells * K / (ms64 * 1e-3)
    log(f"FP64: {ms64 / K:.4f} ms/step, {rate64:.4g} cell-updates/s ({t64}, dt*rho {info64['dt_rho_max']:.3f}, "
        f"{info64['seg_rows']} rows per segment)")
    roof64 = profile_pass(w, F.FP64, args.profile_steps, jg, info64["seg_rows"], 0, info64["store_policy"],
                          info64["tile_order"])
    log(f"FP64 stage kernel: {roof64['avg_launch_us']} us/launch, {roof64['achieved']} GB/s ({roof64['frac'] * 100:.1f}% of HBM)")
    psi32, ms32, t32, info32 = run_graph_path(w, F.FP32C, K, W, jg, args.seg_rows_fp32c)
    rate32 = cells * K / (ms32 * 1e-3)
    roof32 = profile_pass(w, F.FP32C, args.profile_steps, jg, info32["seg_rows"], info32["seg_rows_axis"],
                          info32["store_policy"], info32["tile_order"])
    errs = fp32c_errors(w, psi64, psi32)
    del psi32
    torch.cuda.empty_cache()
    # the increment form takes the FP32C plan's tuned segment length (no second autotuning)
    psi32i, ms32i, t32i, info32i = run_graph_path(w, F.FP32C, K, W, jg, args.seg_rows_fp32c or info32["seg_rows"],
                                                  extra_flags=F.PLAN_INCREMENT_FORM,
                                                  store_policy=info32["store_policy"], tile_order=info32["tile_order"])
    rate32i = cells * K / (ms32i * 1e-3)
    errs_i = fp32c_errors(w, psi64, psi32i)
    del psi64, psi32i
    torch.cuda.empty_cache()
    log(f"FP32C increment form: {ms32i / K:.4f} ms/step, {rate32i:.4g} cell-updates/s "
        f"({info32i['launches_per_step']} launches per step), errors after {W + K} steps {errs_i}")
    log(f"FP32C: {ms32 / K:.4f} ms/step, {rate32:.4g} cell-updates/s, stage kernel {roof32['avg_launch_us']} us "
        f"({roof32['frac'] * 100:.1f}%), errors after {W + K} steps {errs}")
    fp32c = dict(value=rate32, ms_per_step=ms32 / K, dtype="f32+comp", vs_fp64=rate32 / rate64, roofline=roof32,
                 error_vs_fp64_after_steps=W + K, **errs,
                 tiling=dict(seg_rows=info32["seg_rows"], seg_rows_axis=info32["seg_rows_axis"],
                             store_policy=info32["store_policy"], tile_order=info32["tile_order"],
                             autotune_ms=round(info32["autotune_ms"], 1)),
                 **t32)
    fp32c_inc = dict(value=rate32i, ms_per_step=ms32i / K, dtype="f32+comp, increment form", vs_fp64=rate32i / rate64,
                     vs_fp32c=rate32i / rate32, launches_per_step=info32i["launches_per_step"],
                     error_vs_fp64_after_steps=W + K, **errs_i, **t32i)

    full = None
    if args.full_steps > 0 and not args.headline_only:
        res, psis = {}, {}
        for pt, prec, seg, fl in (("fp64", F.FP64, args.seg_rows_fp64, 0), ("fp32c", F.FP32C, args.seg_rows_fp32c, 0),
                                  ("fp32c_increment", F.FP32C, args.seg_rows_fp32c, F.PLAN_INCREMENT_FORM)):
            psi, ms, tt, info = run_graph_path(w, prec, args.full_steps, 0, jg, seg, extra_flags=fl)
            res[pt] = dict(value=cells * args.full_steps / (ms * 1e-3), ms_per_step=ms / args.full_steps, **tt)
            psis[pt] = psi
            log(f"full length {pt}: {args.full_steps} steps, {ms / args.full_steps:.3f} ms/step, "
                f"{res[pt]['value']:.4g} cell-updates/s ({tt})")
        full = dict(steps=args.full_steps, graph=True, fp64=res["fp64"], fp32c=res["fp32c"],
                    fp32c_increment=res["fp32c_increment"],
                    fp32c_vs_fp64=res["fp32c"]["value"] / res["fp64"]["value"],
                    fp32c_error_vs_fp64=fp32c_errors(w, psis["fp64"], psis["fp32c"]),
                    fp32c_increment_vs_fp64=res["fp32c_increment"]["value"] / res["fp64"]["value"],
                    fp32c_increment_error_vs_fp64=fp32c_errors(w, psis["fp64"], psis["fp32c_increment"]))
        log(f"full length FP32C error vs FP64 after {args.full_steps} steps: {full['fp32c_error_vs_fp64']}; "
            f"increment form {full['fp32c_increment_error_vs_fp64']}")
        del psis, psi
        torch.cuda.empty_cache()

    extra = {}
    if not args.headline_only:
        extra["sources"] = sources_pass(w, smp)
        del smp
        torch.cuda.empty_cache()
        if args.current_driven_steps > 0:
            extra["current_driven"] = graph_workload_pass(I.current_driven(), args.current_driven_steps, W, "current-driven")
        if args.batched_steps > 0:
            extra["batched"] = graph_workload_pass(I.batched_uneven(), args.batched_steps, W,
                                                   "batched, default grouping")
            extra["batched_per_width"] = graph_workload_pass(I.batched_uneven(), args.batched_steps, W,
                                                             "batched, one launch batch per width",
                                                             F.PLAN_PER_WIDTH)
            extra["batched_mixed_widths"] = graph_workload_pass(I.batched_uneven(), args.batched_steps, W,
                                                                "batched, one launch batch for all widths",
                                                                F.PLAN_MIXED_WIDTHS)
        if args.envelope_steps > 0:
            extra["envelope"] = envelope_pass(args.envelope_steps)
        if args.correction_steps > 0:
            extra["correction"] = correction_pass(args.correction_steps, W)
    cpu = None if args.no_cpu else cpu_baseline(w)
    if cpu:
        log(f"CPU oracle: {cpu['value']:.4g} cell-updates/s on {cpu['cores']} threads, "
            f"{cpu['one_core']['value']:.4g} on one core ({cpu['cpu_model']})")
    out = {
        "metric": METRIC, "value": rate64, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms64 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "modes": w.m, "nz": w.nz[0], "nr": w.nr[0], "fd_order": w.fd_order[0],
                   "taylor_order": w.taylor_order, "dt_over_dz": 0.5, "dz_um": 0.032, "dr_um": 0.16,
                   "current": f"{N_SAMPLES} bunch samples at c, J_z deposited every step in the graph",
                   "graph": True, "parallelism": "single GPU, modes batched in one plan"},
        "roofline": roof64,
        "cpu_baseline": cpu,
        "tiling": dict(seg_rows=info64["seg_rows"], store_policy=info64["store_policy"],
                       tile_order=info64["tile_order"], autotune_ms=round(info64["autotune_ms"], 1)),
        "launches_per_step": info64["launches_per_step"],
        "fp32c": fp32c,
        "fp32c_increment": fp32c_inc,
        "full_length": full,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
