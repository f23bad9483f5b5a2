"""Benchmark of the MI355X per-cell update (one GPU).

Timed workload (the `value`): plain hydro, FP64, one 256^3 box + 4 ghost
layers, planar discontinuity of seeded orientation with 1% density noise,
outflow boundaries, gamma 1.4, CFL 0.3; one step = one SSP-RK2 hydro step
(flattening, PPM, HLLC, divergence, both stages, ghost fills, CFL dt of the
next step fused into stage 2).  Inputs are resident in HBM before timing.

Also reported on the same line: the radiation-hydrodynamics step at 256^3
(hydro step + 10 radiation substeps + coupling), the mixed-precision forms
with their L1 / L-inf error against the FP64 path, the batched level step,
the roofline of the dominant kernel measured with HIP events on its stream,
and the FP64 oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "cell updates/s (hydro, RHD) 256^3 on 1 MI355X; % of HBM roofline; FP32 err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (FMA counted as two)
HYDRO_BYTES_PER_CELL_STEP = 200.0  # stage 1: read 40 + write 40; stage 2: read 80 + write 40 (FP64)
# FP64 operations (add, sub, mul, min, max, div, sqrt each one) of one cell in
# one fused RK stage, as the method states them, each interface and cell
# counted once: PPM 45 x 15 (5 variables, 3 axes; the flattening blend, an
# identity where chi = 1, is not counted), HLLC 106 x 3 faces, conserved ->
# primitive 13, flux differences and RK update 57.5 (mean of the stages), CFL
# signal of stage 2 11 (mean).
HYDRO_FLOPS_PER_CELL_STAGE = 45 * 15 + 106 * 3 + 13 + 57.5 + 11
# HBM bytes per stage launch (mean of stages 1 and 2) from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs, scaled by the counts of a plain 2 GiB copy
# (profiles/hydro_fp64_256_counters.md).  Valid only while the kernel sources
# and launch plan are the ones that were measured: reported as null once they change.
# The same runs give the stage's VALU issue rate (SQ_INSTS_VALU against 1024
# SIMDs x 2.4 GHz / 4 cycles per wave64 instruction, mean of the two stages).
STAGE_VALU_ISSUE_FRAC = 0.591
STAGE_TRAFFIC = {"bytes_per_launch": 2.897e9, "sources_sha1": "ab30b73ea0a22e3b6f2c6abed611d3e81d768cd7"}
# The stage kernel's sources and its launch plan (the z-chunk length changes the traffic).
KERNEL_SOURCES = ("paper_2110_01792_amd/csrc/hydro_kernels.hpp", "paper_2110_01792_amd/csrc/qk_device.hpp",
                  "paper_2110_01792_amd/csrc/api.hip")


def counters_valid():
    """True while the kernel sources are the ones the counters were taken on."""
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == STAGE_TRAFFIC["sources_sha1"]


def measured_traffic():
    return STAGE_TRAFFIC["bytes_per_launch"] if counters_valid() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(step, k, torch):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(k):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_hydro(ctx, qb, inputs, torch, steps, warmup, dtype, workload="shock"):
    b, U, p = inputs.hydro_shock(n=256) if workload == "shock" else inputs.sedov(n=256)
    Ud = torch.from_numpy(U).to(dtype).cuda()
    del U
    ctx.fill_ghosts(b, Ud)
    hp = qb.hydro_params(p["gamma"], p["cfl"])
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.compute_dt(b, Ud, hp=hp, dt_dev=dt, host=False)
    step = lambda: ctx.hydro_step(b, Ud, hp, dt_dev=dt, dt_next_dev=dt)
    for _ in range(warmup):
        step()
    ms = timed_steps(step, steps, torch)
    st = ctx.sync_status()
    # second pass with per-kernel events for the roofline
    ctx.timing(True)
    for _ in range(steps):
        step()
    stage_ms, nst = ctx.kernel_time(qb.K_HYDRO_STAGE)
    flat_ms, nfl = ctx.kernel_time(qb.K_FLATTEN)
    ghost_ms, ngh = ctx.kernel_time(qb.K_GHOST)
    ctx.timing(False)
    ncell = b.ncells
    scale = 1.0 if dtype == torch.float64 else 0.5
    out = {
        "ms_per_step": ms / steps,
        "cell_updates_per_s": ncell * steps / (ms * 1e-3),
        "status": int(st),
        "stage_ms_avg": stage_ms / max(nst, 1),
        "flatten_ms_avg": flat_ms / max(nfl, 1),
        "ghost_ms_avg": ghost_ms / max(ngh, 1),
        "stage_launches": nst,
        "ncells": ncell,
    }
    # whole step against HBM: algorithmic bytes per cell-update x updates/s
    out["step_hbm_frac"] = HYDRO_BYTES_PER_CELL_STEP * scale * out["cell_updates_per_s"] / (HBM_PEAK_GBS * 1e9)
    # algorithmic bytes per stage launch: average of the two stages
    bytes_per_launch = ncell * HYDRO_BYTES_PER_CELL_STEP * scale / 2.0
    out["stage_achieved_GBs"] = bytes_per_launch / (out["stage_ms_avg"] * 1e-3) / 1e9
    out["stage_achieved_TFLOPs"] = ncell * HYDRO_FLOPS_PER_CELL_STAGE / (out["stage_ms_avg"] * 1e-3) / 1e12
    del Ud
    torch.cuda.empty_cache()
    return out, b, p


# read E_r, F (32), write 32 (FP64, per cell); the density for the optical
# depths (8 B more) is read only when a face of the step is optically thick,
# which no face of the log-normal workload is
RAD_BYTES_STAGE1 = 64.0
RAD_BYTES_STAGE2 = 168.0   # read Ur1, Ur (64) + gas (40), write Ur (32) + m, E (32)


def bench_rhd(ctx, qb, inputs, torch, steps, warmup, dtype, n=256, recon=0, closure=0, source=False):
    b, Ug, Ur, p = inputs.rhd_lognormal(n=n)
    p = dict(p, recon=recon, closure=closure)
    G = torch.from_numpy(Ug).to(dtype).cuda()
    R = torch.from_numpy(Ur).to(dtype).cuda()
    del Ug, Ur
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    J = None
    if source:  # seeded per-cell radiation source rate, uniform in [0, 200)
        gen = torch.Generator(device="cpu").manual_seed(7)
        J = (200.0 * torch.rand(tuple(b.shape), generator=gen, dtype=torch.float64)).to(dtype).cuda()
    rp = qb.rad_params(p, source=J)
    step = lambda: ctx.rhd_step(b, G, R, rp)
    for _ in range(warmup):
        step()
    G0, R0 = G.clone(), R.clone()  # state at the first timed step
    ms = timed_steps(step, steps, torch)
    st = ctx.sync_status()
    # Second pass over the same steps (the path is deterministic): per-kernel
    # HIP events, and the substep count N of every step (N = ceil(dt_h / dt_r)
    # <= nsub_max follows the hydro dt, so it changes as the flow develops;
    # launches for substeps beyond N return at once and are not counted as work).
    G.copy_(G0)
    R.copy_(R0)
    del G0, R0
    ctx.newton_iter_max()
    hp = qb.hydro_params(p["gamma"], p["cfl"], recon)
    nsub = torch.zeros(1, dtype=torch.int32, device="cuda")
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    ns = []
    ctx.timing(True)
    for _ in range(steps):
        ctx.compute_dt(b, G, hp=hp, rp=rp, dt_dev=dtd, nsub_dev=nsub, host=False)
        ns.append(int(nsub.item()))
        step()
    r1_ms, n1 = ctx.kernel_time(qb.K_RAD_STAGE)
    r2_ms, n2 = ctx.kernel_time(qb.K_RAD_COUPLE)
    hs_ms, nh = ctx.kernel_time(qb.K_HYDRO_STAGE)
    ctx.timing(False)
    it = ctx.newton_iter_max()
    ncell = b.ncells
    scale = 1.0 if dtype == torch.float64 else 0.5
    nact = max(sum(ns), 1)
    nmean = sum(ns) / len(ns)
    out = {"ms_per_step": ms / steps, "cell_updates_per_s": ncell * steps / (ms * 1e-3), "status": int(st),
           "rad_stage1_ms_avg": r1_ms / nact, "rad_stage2_couple_ms_avg": r2_ms / nact,
           "hydro_stage_ms_avg": hs_ms / max(nh, 1), "launches": [n1, n2, nh], "active_substeps": nact,
           "nsub_mean": nmean, "nsub_range": [min(ns), max(ns)], "newton_iter_max": it,
           "ncells": ncell, "reconstruction": "PLM" if recon == 1 else "PPM",
           "closure": ("Levermore", "Eddington", "Minerbo")[closure], "source": bool(source)}
    # algorithmic bytes of a step with the mean substep count of the timed steps
    rhd_bytes = HYDRO_BYTES_PER_CELL_STEP + nmean * (RAD_BYTES_STAGE1 + RAD_BYTES_STAGE2)
    out["bytes_per_cell_step"] = rhd_bytes * scale
    out["step_hbm_frac"] = rhd_bytes * scale * out["cell_updates_per_s"] / (HBM_PEAK_GBS * 1e9)
    out["rad_stage1_achieved_GBs"] = ncell * RAD_BYTES_STAGE1 * scale / (out["rad_stage1_ms_avg"] * 1e-3) / 1e9
    out["rad_stage2_achieved_GBs"] = ncell * RAD_BYTES_STAGE2 * scale / (out["rad_stage2_couple_ms_avg"] * 1e-3) / 1e9
    del G, R, J
    torch.cuda.empty_cache()
    return out


def mixed_error_hydro(ctx, qb, inputs, torch, nsteps=20):
    """FP32 path vs FP64 path (the latter matches the oracle to 1e-10 per step)
    on the 256^3 shock box, both from the same FP32-rounded start and the same
    dt sequence: per-variable normalised L1 and relative L-inf."""
    b, U, p = inputs.hydro_shock(n=256)
    U = inputs.to_f32_and_back(U)
    hp = qb.hydro_params(p["gamma"], p["cfl"])
    D = torch.from_numpy(U).cuda()
    F = D.float()
    del U
    ctx.fill_ghosts(b, D)
    ctx.fill_ghosts(b, F)
    dts = []
    for _ in range(nsteps):
        dts.append(ctx.compute_dt(b, D, hp=hp))
        ctx.hydro_step(b, D, hp, dt=dts[-1])
    for dt in dts:
        ctx.hydro_step(b, F, hp, dt=dt)
    torch.cuda.synchronize()
    return error_norms(b, D, F, torch)


def error_norms(b, D, F, torch):
    g = b.ng
    sl = (slice(None), slice(g, g + b.n[2]), slice(g, g + b.n[1]), slice(g, g + b.n[0]))
    d = (F[sl].double() - D[sl]).abs().reshape(D.shape[0], -1)
    o = D[sl].abs().reshape(D.shape[0], -1)
    dens = D[sl][0].abs().sum()
    l1 = (d.sum(1) / torch.where(o.sum(1) > 0, o.sum(1), dens)).cpu().tolist()
    li = (d.max(1).values / torch.where(o.max(1).values > 0, o.max(1).values, D[sl][0].abs().max())).cpu().tolist()
    return {"l1": l1, "linf": li}


def mixed_error_rhd(ctx, qb, inputs, torch, nsteps=20):
    b, Ug, Ur, p = inputs.rhd_lognormal(n=256)
    Ug, Ur = inputs.to_f32_and_back(Ug), inputs.to_f32_and_back(Ur)
    rp = qb.rad_params(p)
    GD, RD = torch.from_numpy(Ug).cuda(), torch.from_numpy(Ur).cuda()
    GF, RF = GD.float(), RD.float()
    del Ug, Ur
    for X in (GD, RD, GF, RF):
        ctx.fill_ghosts(b, X)
    for _ in range(nsteps):
        ctx.rhd_step(b, GD, RD, rp)
        ctx.rhd_step(b, GF, RF, rp)
    torch.cuda.synchronize()
    g = b.ng
    sl = (slice(1, 4), slice(g, g + b.n[2]), slice(g, g + b.n[1]), slice(g, g + b.n[0]))
    scale = p["c"] * RD[0][sl[1:]].abs().sum()
    flux_vs_cE = ((RF[sl].double() - RD[sl]).abs().reshape(3, -1).sum(1) / scale).cpu().tolist()
    return {"gas": error_norms(b, GD, GF, torch), "rad": error_norms(b, RD, RF, torch), "steps": nsteps,
            "rad_flux_l1_over_c_sum_Er": flux_vs_cE,
            "note": "each path takes its own CFL dt (both capped to N_sub,max dt_r, the same value); F starts "
                    "at zero and is bounded by c E_r, so its error is also given against c sum(E_r)"}


def bench_amr(ctx, qb, inputs, torch, steps, warmup, n=256, m=256):
    """Two levels, refinement ratio 2: a periodic n^3 coarse box and an m^3
    fine box over its centre, smooth seeded field, dt held at its initial CFL
    value.  One coarse step = ghost fill, coarse step with a flux register over
    the footprint, two fine half steps with ghosts interpolated from the coarse
    level in space and time, average-down, reflux.  Beside it, the same three
    box steps without the AMR work (plain steps, fine ghosts held fixed)."""
    off = ((n - m // 2) // 2,) * 3
    cb, Uc, fb, Uf, off, hp_d = inputs.two_level(n=n, m=m, off=off, seed=61)
    C = torch.from_numpy(Uc).cuda()
    F = torch.from_numpy(Uf).cuda()
    del Uc, Uf
    hp = qb.hydro_params(hp_d["gamma"], hp_d["cfl"])
    lo = tuple(off)
    hi = tuple(off[d] + fb.n[d] // 2 for d in range(3))
    ctx.fill_ghosts(cb, C)
    ctx.prolong(cb, C, C, 0.0, fb, F, off)
    dt = min(ctx.compute_dt(cb, C, hp=hp), 2.0 * ctx.compute_dt(fb, F, hp=hp))
    C_old = torch.empty_like(C)
    reg_c = torch.zeros(qb.region_size(lo, hi), dtype=torch.float64, device="cuda")
    reg_f = torch.zeros(qb.region_size((0, 0, 0), fb.n), dtype=torch.float64, device="cuda")

    def amr_step():
        ctx.fill_ghosts(cb, C)
        C_old.copy_(C)
        reg_c.zero_()
        reg_f.zero_()
        ctx.hydro_step_reg(cb, C, hp, lo, hi, reg_c, dt=dt)
        for alpha in (0.0, 0.5):
            ctx.prolong(cb, C_old, C, alpha, fb, F, off)
            ctx.hydro_step_reg(fb, F, hp, (0, 0, 0), fb.n, reg_f, dt=0.5 * dt)
        ctx.average_down(fb, F, cb, C, off)
        ctx.reflux(cb, C, lo, hi, reg_c, fb, reg_f)

    def plain_steps():
        ctx.hydro_step(cb, C, hp, dt=dt)
        for _ in range(2):
            ctx.hydro_step(fb, F, hp, dt=0.5 * dt)

    for _ in range(warmup):
        amr_step()
    ms = timed_steps(amr_step, steps, torch)
    st = ctx.sync_status()
    ms_plain = timed_steps(plain_steps, steps, torch)
    st = st or ctx.sync_status()
    updates = cb.ncells + 2 * fb.ncells
    out = {"ms_per_coarse_step": ms / steps, "cell_updates_per_s": updates * steps / (ms * 1e-3),
           "status": int(st), "coarse_cells": cb.ncells, "fine_cells": fb.ncells,
           "plain_ms_same_box_steps": ms_plain / steps, "amr_overhead": ms / ms_plain - 1.0,
           "workload": "hydro FP64, periodic %d^3 coarse box, %d^3 fine box (ratio 2) over coarse cells "
                       "[%d, %d)^3, smooth seeded field (gamma 5/3), dt fixed at its initial CFL 0.3 value; "
                       "updates = coarse cells + 2 x fine cells per coarse step" % (n, m, lo[0], hi[0])}
    del C, F, C_old
    torch.cuda.empty_cache()
    return out


def bench_batch(ctx, qb, inputs, torch, steps, dtype):
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=600, seed=5)
    G = [torch.from_numpy(u).to(dtype).cuda() for u in Ugs]
    R = [None if u is None else torch.from_numpy(u).to(dtype).cuda() for u in Urs]
    ncell = sum(b.ncells for b in boxes)
    nrad = sum(1 for u in Urs if u is not None)
    del Ugs, Urs
    hpp, rp = qb.hydro_params(hp["gamma"], hp["cfl"]), qb.rad_params(p)
    t0 = time.perf_counter()
    ctx.batch_step(boxes, G, R, hpp, rp)  # tunes, captures, runs once
    build_s = time.perf_counter() - t0
    tile, zc, tune_ms = ctx.batch_config()
    step = lambda: ctx.batch_step(boxes, G, R, hpp, rp, host_dt=False)
    step()
    ms = timed_steps(step, steps, torch)
    st = ctx.sync_status()
    del G, R
    torch.cuda.empty_cache()
    return {"ms_per_step": ms / steps, "cell_updates_per_s": ncell * steps / (ms * 1e-3), "status": int(st),
            "boxes": len(boxes), "rad_boxes": nrad, "cells": ncell, "tile": tile, "zc": zc,
            "first_call_s": build_s,
            "workload": "600 boxes, edges per axis from {8,16,24,32,48,64}, half RHD (10 substeps), fixed ghosts; "
                        "one graph replay per level step"}


def environment(torch):
    from paper_2110_01792_amd import build as pb
    props = torch.cuda.get_device_properties(0)
    return {"device": torch.cuda.get_device_name(0), "arch": getattr(props, "gcnArchName", "unknown"),
            "compute_units": props.multi_processor_count, "hip": torch.version.hip, "torch": torch.__version__,
            "library_flags": "hipcc --offload-arch=%s %s" % (pb.ARCH, " ".join(pb.FLAGS)),
            "timing": "device synchronised, HIP events around the timed steps on the stream the library "
                      "launches on, device synchronised; no host synchronisation inside (dt and N_sub stay on "
                      "the device); per-kernel averages from the library's own HIP events in a second pass"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_hydro(inputs, oracle, steps=3):
    """The oracle on the host cores: `steps` FP64 hydro steps of the full 256^3
    benchmark box on all threads, then one step on a single thread."""
    b, U, p = inputs.hydro_shock(n=256)
    threads = oracle.set_threads(0)
    oracle.fill_ghosts(b, U)
    t0 = time.perf_counter()
    for _ in range(steps):
        oracle.hydro_step(b, U, p["gamma"], p["cfl"])
    t = time.perf_counter() - t0
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.hydro_step(b, U, p["gamma"], p["cfl"])
    t1 = time.perf_counter() - t1
    oracle.set_threads(0)
    return {"value": steps * b.ncells / t, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d FP64 hydro steps of the full 256^3 benchmark box on %d threads (%.1f s)" % (steps, threads, t),
            "value_1_thread": b.ncells / t1,
            "sample_1_thread": "one further step on 1 thread (%.1f s)" % t1,
            "cpu_model": cpu_model()}


def run_only(args, torch, qb, inputs):
    """One section, printed as its own JSON line (profiling aid)."""
    if args.only == "copy":
        n = 2 ** 31 // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.warmup + args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"section": "copy", "bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                          "launches": args.warmup + args.steps}), flush=True)
        return
    ctx = qb.Context(0)
    f64, f32 = torch.float64, torch.float32
    if args.only in ("hydro", "hydro32"):
        out, _, _ = bench_hydro(ctx, qb, inputs, torch, args.steps, args.warmup, f64 if args.only == "hydro" else f32)
    elif args.only == "sedov":
        out, _, _ = bench_hydro(ctx, qb, inputs, torch, args.steps, args.warmup, f64, workload="sedov")
    elif args.only in ("rhd", "rhd32"):
        out = bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, f64 if args.only == "rhd" else f32)
    elif args.only == "rhdplm":
        out = bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, f64, recon=1)
    elif args.only == "rhdvar":
        out = {"eddington": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, f64, closure=1),
               "minerbo": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, f64, closure=2),
               "source": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, f64, source=True)}
    elif args.only == "amr":
        out = bench_amr(ctx, qb, inputs, torch, args.steps, args.warmup)
    elif args.only == "batch32":
        out = bench_batch(ctx, qb, inputs, torch, args.steps, f32)
    else:
        out = bench_batch(ctx, qb, inputs, torch, args.steps, f64)
    ctx.close()
    print(json.dumps({"section": args.only, **out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--only", default="all", choices=["all", "hydro", "rhd", "hydro32", "rhd32", "sedov", "rhdplm", "rhdvar", "amr", "batch", "batch32", "copy"],
                    help="run one section only (for profiler runs); 'copy' runs a plain 2 GiB device copy used "
                         "to calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py runs on one GPU only: the update is measured on one GPU's 256^3 share; "
            "the library has no multi-GPU halo exchange (--gpus must be 1)")
        sys.exit(2)

    import torch
    from paper_2110_01792_amd import binding as qb
    from paper_2110_01792_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only != "all":
        return run_only(args, torch, qb, inputs)
    ctx = qb.Context(0)
    log("hydro FP64 256^3 ...")
    h64, b, p = bench_hydro(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64)
    log("hydro FP64:", h64)
    log("RHD FP64 256^3 ...")
    r64 = bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64)
    log("RHD FP64:", r64)
    log("paper workloads: Sedov 256^3 PPM hydro, RHD 256^3 PLM ...")
    sed64, _, _ = bench_hydro(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64, workload="sedov")
    plm64 = bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64,
                      recon=1)
    log("Sedov:", sed64, "RHD PLM:", plm64)
    log("closures, source term, two-level AMR ...")
    variants = {
        "rhd_eddington_f64": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64, closure=1),
        "rhd_minerbo_f64": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64, closure=2),
        "rhd_source_f64": bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float64, source=True),
        "amr_two_level_f64": bench_amr(ctx, qb, inputs, torch, args.steps, args.warmup),
    }
    log("variants:", variants)
    log("mixed ...")
    h32, _, _ = bench_hydro(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float32)
    r32 = bench_rhd(ctx, qb, inputs, torch, args.steps, args.warmup, torch.float32)
    h32["error_vs_f64_20_steps"] = mixed_error_hydro(ctx, qb, inputs, torch)
    r32["error_vs_f64"] = mixed_error_rhd(ctx, qb, inputs, torch)
    log("mixed hydro:", h32)
    log("mixed RHD:", r32)
    log("batched ...")
    b64 = bench_batch(ctx, qb, inputs, torch, args.steps, torch.float64)
    b32 = bench_batch(ctx, qb, inputs, torch, args.steps, torch.float32)
    log("batch:", b64, b32)

    # Headline roofline: the dominant kernel (the fused hydro RK stage) against
    # the HBM roofline, the bound the method's measurement plan names;
    # achieved = the stage's algorithmic bytes per launch / its mean launch
    # time from HIP events on its stream.  The stage is in fact limited by
    # FP64 vector issue (about 1075 FP64 operations per 100 B, above the ridge
    # of 78.6 TF/s / 8 TB/s): that figure is given beside it, against the
    # FMA peak (78.6) and the peak without FMA (39.3, each operation one
    # instruction).
    stage_tf = h64["stage_achieved_TFLOPs"]
    roof = {
        "bound": "hbm",
        "achieved": round(h64["stage_achieved_GBs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(h64["stage_achieved_GBs"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(),
        "traffic_unit": "HBM bytes per stage launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated; "
                        "null when the kernel sources differ from those the counters were taken on)",
        "kernel": "stage_kernel<double,double,1|2> (fused hydro RK stage, 16x14 tiles)",
        # the counted bytes over the same launch time: the HBM fraction the
        # stage actually moves (halo re-reads included)
        "traffic_frac": (round(measured_traffic() / (h64["stage_ms_avg"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
                         if measured_traffic() is not None else None),
        "bytes_per_cell_launch": HYDRO_BYTES_PER_CELL_STEP / 2,
        "cells_per_launch": h64["ncells"],
        "stage_ms_avg": round(h64["stage_ms_avg"], 4),
        "step_hbm_frac": round(h64["step_hbm_frac"], 4),
        "fp64_issue": {
            "flops_per_cell_launch": HYDRO_FLOPS_PER_CELL_STAGE,
            "achieved_TFLOPs": round(stage_tf, 3),
            "frac_of_fma_peak_78.6": round(stage_tf / FP64_PEAK_TFLOPS, 4),
            "frac_of_no_fma_peak_39.3": round(stage_tf / (FP64_PEAK_TFLOPS / 2), 4),
            "valu_issue_frac": STAGE_VALU_ISSUE_FRAC if counters_valid() else None,
            "note": "algorithmic FP64 operations (each add, mul, min, max, div, sqrt one) per cell and stage; "
                    "valu_issue_frac = SQ_INSTS_VALU of the same kernel against the chip's wave64 issue slots "
                    "(profiles/hydro_fp64_256_counters.md), null when the sources changed since",
        },
        "rhd_step_hbm_frac": round(r64["step_hbm_frac"], 4),
    }
    line = {
        "metric": METRIC,
        "value": h64["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hydro FP64, one 256^3 box + 4 ghost layers, planar discontinuity (seeded "
                               "orientation, rho 1/0.125, P 1/0.1) + 1% density noise, outflow, gamma 1.4, "
                               "CFL 0.3; PPM + flattening + HLLC + SSP-RK2",
                   "cells": h64["ncells"], "seed": 2},
        "roofline": roof,
        "hydro_f64": h64,
        "rhd_f64": dict(r64, workload="RHD FP64 256^3 periodic, log-normal density, T_gas and T_rad U[0.5,2], "
                                       "chat = 10 max c_s, kappa 1, Levermore, Newton tol 1e-12; one step = hydro "
                                       "RK2 + 10 radiation RK2 substeps + coupling"),
        "paper_workloads": {
            "sedov_ppm_f64": dict(sed64, workload="Sedov blast 256^3 periodic, rho 1, P 10 in r < 0.1 else 0.1, "
                                                   "gamma 5/3, CFL 0.25, PPM (the paper's hydro performance "
                                                   "problem)",
                                  paper_context="113.34 Mzones/s V100, 254.05 Mzones/s A100 (PPM, 128^3 boxes)"),
            "rhd_plm_f64": dict(plm64, workload="RHD FP64 256^3 as rhd_f64 with PLM for hydro and radiation",
                                paper_context="22.55 Mzones/s V100, 39.04 Mzones/s A100 (PLM, radiation-driven "
                                              "shell 256^3, 10 substeps)"),
        },
        "variants": variants,
        "hydro_mixed": h32,
        "rhd_mixed": r32,
        "batch_f64": b64,
        "batch_mixed": b32,
        "environment": environment(torch),
    }
    if not args.no_cpu:
        import oracle
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline_hydro(inputs, oracle)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
