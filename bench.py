"""Benchmark: grid-point updates per second of the 2D acoustic hot path.

Workload (the paper's acoustic system at production size): 4096 x 4096
periodic grid, 4th-order staggered stencil, 4-layer medium (c in [1.5, 4.5],
rho in [1.0, 2.5]), CFL 0.4, four Gaussian pressure pulses, 10000 leapfrog
steps by default; synthetic, seeded inputs.  A "step" is one full leapfrog
step of the whole grid (both half-steps, every field, the solution update
of Alg. 1 or Alg. 2); the discrete energy is computed in fp64 every 1000
steps inside the timed region.

The headline value is fp16 storage with the 6-operation compensated update
(TwoSum); fp32, plain fp16 and plain bf16 run on the same workload for
comparison.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "grid-point updates/s (FP16+comp vs FP32) at fixed energy drift; p50/p99 latency"
ENERGY_EVERY = 1000

# Algorithmic HBM bytes per cell and step of the fused acoustic kernel: every
# field (vx, vy, p) and, with compensation, every compensation term read and
# written once, the two fp32 material arrays (b, kappa) read once.
def bytes_per_cell(storage: str, comp: str) -> int:
    """Algorithmic bytes per cell and step of the 2D step: three fields read
    and written, their compensation terms (a storage-format value, or one
    byte with 8-bit words) read and written, two fp32 material arrays read."""
    e = 4 if storage == "f32" else 2
    fields = 3 * e * 2
    comps = {"none": 0, "twosum8": 3 * 1 * 2}.get(comp, 3 * e * 2)
    return fields + comps + 2 * 4


VARIANTS = [("f16", "twosum"), ("f32", "none"), ("f16", "none"), ("bf16", "none"),
            ("f16", "twosum8")]


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in ("acoustic2d.hip", "acoustic2d_tb.hip", "acoustic2d_tb.h", "acoustic2d_kernels.h",
                 "hw_device.h", "hw_internal.h"):
        with open(os.path.join(ROOT, "paper_2310_00236_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(tag: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_acoustic2d_4096_o4.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_digest():
        return None
    v = rec.get("variants", {}).get(tag)
    return None if v is None else v.get("hbm_bytes_per_launch")


def window_drift(energy, steps, first, last):
    """Relative energy drift max |E_n - E_first| / E_first over the samples
    taken from step `first` to step `last`; None with fewer than two."""
    sel = (steps >= first) & (steps <= last)
    e = energy[sel]
    if len(e) < 2:
        return None
    return float(np.max(np.abs(e - e[0])) / abs(e[0]))


def steps_per_launch(hw, tile) -> int:
    """Time steps one launch of 2D tile shape `tile` advances (the
    temporally blocked kinds 4 and 5 advance two)."""
    return 2 if hw.tiles("acoustic2d")[tile][3] in (4, 5) else 1


def run_variant(hw, torch, w, storage, comp, steps, warmup, tile):
    pb = hw.Problem("acoustic2d", w.nx, w.ny, 1, w.order, storage, comp, w.dx,
                    w.dt, 0, (warmup + steps) // ENERGY_EVERY + 8)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([w.rho, w.kappa])
    plan.set_fields(w.fields())
    stream = torch.cuda.current_stream()
    plan.advance(warmup, ENERGY_EVERY)
    # energy at the start and at the end of the timed window, recorded
    # outside the events; inside, every ENERGY_EVERY steps
    plan.record_energy()
    start = plan.step
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    plan.advance(steps, ENERGY_EVERY)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    plan.record_energy()
    end = plan.step
    # average duration of the step kernel alone: back-to-back launches with
    # no energy evaluation in between, bracketed by events on the same stream
    nk = min(200, max(steps, 1))
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    plan.advance(nk, 0)
    k1.record(stream)
    torch.cuda.synchronize()
    kernel_ms = k0.elapsed_time(k1) / nk
    energy, esteps = plan.energy_trace()
    plan.close()
    cells = w.nx * w.ny
    per = steps_per_launch(hw, tile)
    # a launch reads and writes the state once: per step, its bytes divided
    # by the steps it advances
    bpc = bytes_per_cell(storage, comp) / per
    return {
        "glups": cells * steps / (ms * 1e-3) / 1e9,
        "ms_per_step": ms / steps,
        "wall_s": wall,
        "kernel_ms": kernel_ms,
        "steps_per_launch": per,
        "energy_drift_window": window_drift(energy, esteps, start, end),
        "energy_samples_window": int(np.sum((esteps >= start) & (esteps <= end))),
        "bytes_per_cell": bpc,
        "hbm_gbs_algorithmic": bpc * cells / (kernel_ms * 1e-3) / 1e9,
    }


LAYERED_GOLDEN = os.path.join(ROOT, "tests", "golden", "layered4096_fp64_energy.csv")


def read_layered_golden(path=LAYERED_GOLDEN):
    """The FP64 oracle's energy of the 4096^2 layered workload by rounded
    start ('f16', 'f32', 'bf16') and step, or {} if it is missing."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if line.startswith("#"):
            continue
        start, step, e = line.strip().split(",")
        out.setdefault(start, {})[int(step)] = float(e)
    return out


def drift_run(hw, w, storage, comp, tile, nsteps, ref):
    """The workload's full run (untimed): energy every ENERGY_EVERY steps,
    compared with the FP64 oracle's energy from the same rounded start.  The
    oracle conserves its energy to roundoff (pinned), so where its stored
    record has no entry for a step its starting energy stands for it."""
    pb = hw.Problem("acoustic2d", w.nx, w.ny, 1, w.order, storage, comp, w.dx,
                    w.dt, 0, nsteps // ENERGY_EVERY + 2)
    plan = hw.Plan(pb)
    plan.set_tile(tile)
    plan.set_material([w.rho, w.kappa])
    plan.set_fields(w.fields())
    plan.advance(nsteps, ENERGY_EVERY)
    energy, esteps = plan.energy_trace()
    plan.close()
    out = {"steps": nsteps, "energy_samples": int(len(energy)),
           "energy_drift_self": float(np.max(np.abs(energy - energy[0])) / energy[0])}
    if ref:
        e_ref = np.array([ref.get(int(n), ref[0]) for n in esteps])
        out["energy_drift_vs_fp64"] = float(np.max(np.abs(energy - e_ref)) / ref[0])
        out["fp64_reference_steps"] = sorted(n for n in ref if n <= nsteps)
    else:
        out["energy_drift_vs_fp64"] = None
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, target_s=12.0):
    """The FP64 oracle (fp64 storage and stencil, plain update: the
    reference solver) on the same 4096^2 workload from its initial state,
    with all of the oracle's threads and with one thread, each for about
    target_s seconds of whole steps (a one-step call first sizes the run;
    each call's set-up is included in its time)."""
    import oracle
    f0 = w.fields()
    args = (w.nx, w.ny, w.order, w.dx, w.dt, w.rho, w.kappa)

    def rate(threads):
        t = time.perf_counter()
        f, _, _ = oracle.acoustic2d(*args, f0, storage="f64", stencil="f64", comp="none",
                                    nsteps=1, nthreads=threads)
        t1 = time.perf_counter() - t
        steps = max(1, int(target_s / t1))
        t = time.perf_counter()
        oracle.acoustic2d(*args, f, storage="f64", stencil="f64", comp="none",
                          nsteps=steps, nthreads=threads)
        secs = time.perf_counter() - t
        return w.nx * w.ny * steps / secs / 1e9, steps, secs

    nthreads = oracle.max_threads()
    g_all, n_all, s_all = rate(0)
    g_one, n_one, s_one = rate(1)
    return {"value": g_all, "unit": "GLUPS", "cores": nthreads, "kind": "oracle",
            "sample": f"{n_all} steps of the {w.nx}x{w.ny} order-4 layered workload "
                      f"({s_all:.1f} s, {nthreads} threads); one thread: {n_one} steps "
                      f"({s_one:.1f} s)",
            "arithmetic": "fp64 storage, fp64 stencil, plain update (the FP64 reference)",
            "single_thread_value": g_one,
            "nproc": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}


ELASTIC_BYTES_ALGO = {"f32+none": 84, "f16+twosum": 84, "f16+none": 48}
ELASTIC_BYTES_TWO_PASS = {"f32+none": 120, "f16+twosum": 120, "f16+none": 60}


def elastic_source_digest() -> str:
    h = hashlib.sha256()
    for name in ("elastic3d.hip", "hw_device.h", "hw_internal.h"):
        with open(os.path.join(ROOT, "paper_2310_00236_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic3d(tag: str):
    """HBM bytes per launch of the 3D step kernel from the committed
    rocprofv3 counter summary, if it was taken on the current source."""
    path = os.path.join(ROOT, "profiles", "traffic_elastic3d_512.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != elastic_source_digest():
        return None
    v = rec.get("variants", {}).get(tag)
    return None if v is None else v.get("hbm_bytes_per_launch")


def run_elastic(hw, torch, n, steps, warmup, variants):
    """3D elastic velocity-stress workload: n^3 periodic, smooth random
    rho/lambda/mu (ratio <= 3), CFL 0.3, explosive Gaussian source on the
    normal stresses."""
    import workloads
    from paper_2310_00236_amd import tuning
    w = workloads.smooth3d(n, nsteps=steps)
    every = max(steps // 10, 1)
    out = {}
    shapes = hw.tiles("elastic3d")
    for storage, comp in variants:
        key = f"{storage}+{comp}"
        pb = hw.Problem("elastic3d", n, n, n, 2, storage, comp, w.dx, w.dt, 0,
                        (steps + warmup) // every + 8)
        plan = hw.Plan(pb)
        tile = tuning.best_tile("elastic3d", 2, storage, comp, n, n, n)
        plan.set_tile(tile)
        plan.set_material([w.rho, w.lam, w.mu])
        plan.set_fields(w.fields())
        stream = torch.cuda.current_stream()
        plan.record_energy()
        plan.advance(warmup, every)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        plan.advance(steps, every)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        plan.record_energy()
        # the step kernel alone: back-to-back launches, no energy in between
        nk = 20
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        plan.advance(nk, 0)
        k1.record(stream)
        torch.cuda.synchronize()
        kernel_ms = k0.elapsed_time(k1) / nk
        energy, _ = plan.energy_trace()
        plan.close()
        cells = n ** 3
        step_ms = ms / steps
        out[key] = {
            "glups": cells * steps / (ms * 1e-3) / 1e9,
            "ms_per_step": step_ms,
            "kernel_ms": kernel_ms,
            "tile": hw.tile_label(shapes[tile]),
            "energy_drift": float(np.max(np.abs(energy - energy[0])) / energy[0]),
            "energy_samples": int(len(energy)),
            "bytes_per_cell_step_algorithmic": ELASTIC_BYTES_ALGO[key],
            "hbm_gbs_algorithmic": ELASTIC_BYTES_ALGO[key] * cells / (kernel_ms * 1e-3) / 1e9,
            "frac_hbm": ELASTIC_BYTES_ALGO[key] * cells / (kernel_ms * 1e-3) / 1e9
            / PEAK_HBM_GBS,
        }
        print(f"# elastic3d {n}^3 {key}: {out[key]}", file=sys.stderr, flush=True)
    res = {"workload": f"elastic3d order-2 {n}^3 periodic, smooth random medium, "
                       f"CFL 0.3, explosive source, {steps} steps",
           "variants": out,
           "vs_f32": out["f16+twosum"]["glups"] / out["f32+none"]["glups"]
           if "f16+twosum" in out and "f32+none" in out else None}
    head = "f16+twosum" if "f16+twosum" in out else next(iter(out))
    h = out[head]
    res["roofline"] = {
        "bound": "hbm", "achieved": h["hbm_gbs_algorithmic"], "peak": PEAK_HBM_GBS,
        "unit": "GB/s", "frac": h["frac_hbm"],
        "traffic": measured_traffic3d(head) if n == 512 else None,
        "kernel": "el3d_fused1_kernel", "variant": head,
        "bytes_per_cell_step": ELASTIC_BYTES_ALGO[head], "cells_per_launch": n ** 3,
        "kernel_ms": h["kernel_ms"]}
    return res


def run_batched(hw, torch, nshots):
    """64 independent layered 2D shots of uneven size and step count, fp16
    with the 6-operation compensated update: one batched launch per step
    (graph-captured runs) against one shot at a time."""
    import workloads
    from paper_2310_00236_amd import tuning
    sizes = workloads.shot_sizes(nshots)
    shots = [workloads.shot(nx, ny, ns, i) for i, (nx, ny, ns) in enumerate(sizes)]
    total = sum(s.nx * s.ny * s.nsteps for s in shots)

    def make():
        plans = []
        for s in shots:
            pb = hw.Problem("acoustic2d", s.nx, s.ny, 1, 4, "f16", "twosum",
                            s.dx, s.dt, 0, 0)
            p = hw.Plan(pb)
            p.set_tile(tuning.best_tile("acoustic2d", 4, "f16", "twosum", s.nx, s.ny))
            p.set_material([s.rho, s.kappa])
            p.set_fields(s.fields())
            plans.append(p)
        return plans

    stream = torch.cuda.current_stream()
    res = {}
    for mode in ("batched", "one_shot_at_a_time"):
        plans = make()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if mode == "batched":
            hw.batch_advance(plans, [s.nsteps for s in shots])
        else:
            for p, s in zip(plans, shots):
                p.advance(s.nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[mode] = {"glups": total / (ms * 1e-3) / 1e9, "seconds": ms * 1e-3}
        for p in plans:
            p.close()
        del plans
        print(f"# batched {mode}: {res[mode]}", file=sys.stderr, flush=True)
    return {"workload": f"{nshots} layered 2D order-4 shots, sides U{{256..2048}}, "
                        f"steps U{{500..5000}}, fp16+TwoSum",
            "cell_steps": total, **res,
            "speedup": res["batched"]["glups"] / res["one_shot_at_a_time"]["glups"]}


PAPER_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                            "golden", "paper2d_ppw10_fp64.csv")
PAPER_VARIANTS = [("f32", "none", "f32"), ("f16", "none", "f32"),
                  ("f16", "fast2sum", "f32"), ("f16", "twosum", "f32"),
                  ("bf16", "none", "f32"), ("bf16", "twosum", "f32"),
                  ("f16", "twosum8", "f32"),
                  # App. B: stencil promoted to fp64, update in fp16; and the
                  # all-fp16 step of Alg. 1 taken literally
                  ("f16", "none", "f64"), ("f16", "fast2sum", "f64"),
                  ("f16", "none", "storage"), ("f16", "fast2sum", "storage")]


def read_paper_golden(path=PAPER_GOLDEN):
    """The FP64 oracle's receiver trace (every 50th step) and energy (every
    500th) of the Sec. 3 experiment, or None if it has not been generated."""
    if not os.path.exists(path):
        return None
    steps, rec, es, ev = [], [], [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            f = line.strip().split(",")
            if f[0] == "E":
                es.append(int(f[1]))
                ev.append(float(f[2]))
            else:
                steps.append(int(f[0]))
                rec.append([float(x) for x in f[1:4]])
    return {"steps": np.array(steps), "rec": np.array(rec),
            "energy_steps": np.array(es), "energy": np.array(ev)}


def trace_rel_l2(trace, gold, col):
    """Relative l2 distance of a receiver record (one value per step) from
    the reference's column col, over the reference rows the run reached;
    None if the reference is still zero there."""
    sel = gold["steps"] <= len(trace)
    ref = gold["rec"][sel, col]
    got = trace[gold["steps"][sel] - 1]
    norm = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / norm) if norm > 0 else None


def run_paper(hw, torch, nsteps=60000):
    """The acoustic experiment of Sec. 3: 600^2 (ppw 10), dt 1e-4, 60000
    steps, Ricker point source on the pressure, one receiver; every storage
    variant on the GPU against the FP64 oracle's receiver trace and energy,
    plus fp32 at ppw 30 as the discretisation reference."""
    import workloads
    from paper_2310_00236_amd import tuning
    gold = read_paper_golden()
    every = 500
    out = {}

    def one(w, storage, comp, stencil="f32"):
        samples = w.source[2]
        pb = hw.Problem("acoustic2d", w.nx, w.ny, 1, w.order, storage, comp, w.dx,
                        w.dt, 0, nsteps // every + 2, src_cap=len(samples),
                        rec_cap=1, rec_steps=nsteps, stencil=stencil)
        plan = hw.Plan(pb)
        # the tuned shape (two steps per launch; plans with another stencil
        # precision step on shape 0 whatever the setting)
        plan.set_tile(tuning.best_tile("acoustic2d", w.order, storage, comp, w.nx, w.ny))
        plan.set_material([w.rho, w.kappa])
        plan.set_fields(w.fields())
        plan.set_source(w.source[0], w.source[1], samples)
        plan.set_receivers(w.receivers)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        plan.advance(nsteps, every)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        rec = plan.receiver_trace()[:, 0, :]
        energy, esteps = plan.energy_trace()
        plan.close()
        return ms, rec, energy, esteps

    w10 = workloads.paper2d(ppw=10, nsteps=nsteps)
    src_end = len(w10.source[2])
    for storage, comp, stencil in PAPER_VARIANTS:
        ms, rec, energy, esteps = one(w10, storage, comp, stencil)
        r = {"glups": w10.cells * nsteps / (ms * 1e-3) / 1e9, "ms_total": ms}
        # energy change once the source has stopped injecting (Sec. 3: flat
        # for a conserving run)
        after = esteps >= src_end + every
        e_after = energy[after]
        # null when the run ends before the source has stopped
        r["energy_change_after_source"] = (
            float((e_after[-1] - e_after[0]) / e_after[0]) if len(e_after) > 1 else None)
        if gold is not None:
            r["p_trace_rel_l2_vs_fp64"] = trace_rel_l2(rec[:, 0], gold, 0)
            ge = np.interp(esteps, gold["energy_steps"], gold["energy"])
            m = esteps >= every
            r["energy_max_rel_dev_vs_fp64"] = float(np.max(np.abs(energy[m] - ge[m]) / ge[m]))
        key = f"{storage}+{comp}" + ("" if stencil == "f32" else f"/stencil-{stencil}")
        out[key] = r
        print(f"# paper2d ppw10 {key}: {r}", file=sys.stderr, flush=True)
    res = {"workload": "acoustic2d order-4 600x600 (ppw 10), dx 1/125, dt 1e-4, rho=c=1, "
                       f"{nsteps} steps, Ricker 5 Hz point source at (200,200), "
                       "receiver at (400,400) (Sec. 3)",
           "reference": "FP64 oracle" if gold is not None else None,
           "variants": out}
    # discretisation reference: fp32 at ppw 30 (same physical positions)
    w30 = workloads.paper2d(ppw=30, nsteps=nsteps)
    ms, rec30, _, _ = one(w30, "f32", "none")
    res["f32_ppw30_glups"] = w30.cells * nsteps / (ms * 1e-3) / 1e9
    if gold is not None:
        res["discretisation_rel_l2_ppw10_vs_ppw30"] = trace_rel_l2(rec30[:, 0], gold, 0)
    print(f"# paper2d ppw30 f32: {res.get('discretisation_rel_l2_ppw10_vs_ppw30')}",
          file=sys.stderr, flush=True)
    return res


APP_A_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                            "golden", "elastic2d_app_a_fp64.csv")
APP_A_VARIANTS = [("f32", "none"), ("f16", "none"), ("f16", "fast2sum"),
                  ("f16", "twosum"), ("bf16", "none"), ("bf16", "twosum")]


def read_app_a_golden(path=APP_A_GOLDEN):
    """The FP64 oracle's receiver record (five fields every 50th step) and
    energy (every 500th) of the App. A experiment, or None."""
    if not os.path.exists(path):
        return None
    steps, rec, es, ev = [], [], [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            f = line.strip().split(",")
            if f[0] == "E":
                es.append(int(f[1]))
                ev.append(float(f[2]))
            else:
                steps.append(int(f[0]))
                rec.append([float(x) for x in f[1:6]])
    return {"steps": np.array(steps), "rec": np.array(rec),
            "energy_steps": np.array(es), "energy": np.array(ev)}


def run_app_a(hw, torch, nsteps=60000, big=4096, big_steps=400):
    """The elastic experiment of App. A: 600^2, free surfaces at the top and
    bottom rows, periodic in x, dt 1e-4, 60000 steps, Ricker source on vy ten
    cells below the surface, one receiver; every storage variant against the
    FP64 oracle's vy record and energy.  Plus the two-pass kernels' rate on
    a big^2 grid of the same medium type (HBM-resident, no source)."""
    import workloads
    from paper_2310_00236_amd import tuning
    gold = read_app_a_golden()
    every = 500
    w = workloads.paper_elastic2d(nsteps=nsteps)
    shapes = hw.tiles("elastic2d")
    samples = w.source[2]
    src_end = len(samples)
    out = {}
    stream = torch.cuda.current_stream()
    for storage, comp in APP_A_VARIANTS:
        pb = hw.Problem("elastic2d", w.nx, w.ny, 1, 2, storage, comp, w.dx, w.dt, 0,
                        nsteps // every + 2, src_cap=len(samples), rec_cap=1,
                        rec_steps=nsteps)
        plan = hw.Plan(pb)
        tile = tuning.best_tile("elastic2d", 2, storage, comp, w.nx, w.ny)
        plan.set_tile(tile)
        plan.set_material([w.rho, w.lam, w.mu])
        plan.set_fields(w.fields())
        plan.set_source(*w.source)
        plan.set_receivers(w.receivers)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        plan.advance(nsteps, every)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        rec = plan.receiver_trace()[:, 0, :]
        energy, esteps = plan.energy_trace()
        plan.close()
        r = {"glups": w.cells * nsteps / (ms * 1e-3) / 1e9, "ms_total": ms,
             "tile": hw.tile_label(shapes[tile])}
        after = esteps >= src_end + every
        e_after = energy[after]
        # null when the run ends before the source has stopped
        r["energy_change_after_source"] = (
            float((e_after[-1] - e_after[0]) / e_after[0]) if len(e_after) > 1 else None)
        if gold is not None:
            r["vy_trace_rel_l2_vs_fp64"] = trace_rel_l2(rec[:, 1], gold, 1)
            ge = np.interp(esteps, gold["energy_steps"], gold["energy"])
            m = esteps >= every
            r["energy_max_rel_dev_vs_fp64"] = float(np.max(np.abs(energy[m] - ge[m]) / ge[m]))
        out[f"{storage}+{comp}"] = r
        print(f"# app_a {storage}+{comp}: {r}", file=sys.stderr, flush=True)
    res = {"workload": f"elastic2d order-2 {w.nx}x{w.ny}, free surfaces on rows 0 and "
                       f"{w.ny - 1}, periodic in x, dx 1/125 km, dt 1e-4 s, {nsteps} steps, "
                       "layered stand-in medium (cs >= 1.0117, cp <= 4.6992 km/s), "
                       "Ricker 5 Hz on vy at (200, 10.5), receiver at (400, 10) (App. A)",
           "reference": "FP64 oracle" if gold is not None else None,
           "variants": out}
    # the two-pass kernels at an HBM-resident size: bytes per cell-step of
    # the two passes: the velocity pass reads 3 stress words, 2 velocity
    # words and b, writes 2 velocity words; the stress pass reads 2 velocity
    # words, 3 stress words and 3 coefficients, writes 3 stress words -> 15
    # words + 4 fp32 coefficients (a word is 4 bytes for fp32 or a 16-bit
    # value with its compensation term, 2 for a plain 16-bit value); one
    # fused pass would need 10 words + 4 coefficients
    rho, lam, mu = workloads.layered_elastic2d(big, big, workloads.seed_for(7, 1))
    cp = float(np.sqrt((lam + 2 * mu) / rho).max())
    dt = 0.5 / cp
    z = np.zeros((big, big))
    f0 = {"sxx": workloads.gaussian2d(big, big, big // 2, big // 2, 8.0)}
    thr = {}
    for storage, comp in (("f32", "none"), ("f16", "twosum"), ("f16", "none")):
        pb = hw.Problem("elastic2d", big, big, 1, 2, storage, comp, 1.0, dt, 0, 0)
        plan = hw.Plan(pb)
        tile = tuning.best_tile("elastic2d", 2, storage, comp, big, big)
        plan.set_tile(tile)
        plan.set_material([rho, lam, mu])
        plan.set_fields({"vx": z, "vy": z, "sxx": f0["sxx"], "syy": z, "sxy": z})
        plan.advance(20)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        plan.advance(big_steps)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / big_steps
        plan.close()
        word = 4 if (storage == "f32" or comp != "none") else 2
        bpc = 15 * word + 4 * 4
        thr[f"{storage}+{comp}"] = {
            "glups": big * big / (ms * 1e-3) / 1e9, "ms_per_step": ms,
            "tile": hw.tile_label(shapes[tile]),
            "bytes_per_cell_step_two_pass": bpc,
            "hbm_gbs_two_pass": bpc * big * big / (ms * 1e-3) / 1e9}
        print(f"# app_a {big}^2 {storage}+{comp}: {thr[f'{storage}+{comp}']}",
              file=sys.stderr, flush=True)
    res[f"throughput_{big}"] = thr
    return res


def run_serving(hw, torch, nreq, glups, budget=None, chunk=200, seed=None):
    """Poisson stream of mixed requests (70% 2D order-4 512^2..4096^2, 30% 3D
    128^3..384^3, 1000..10000 steps, fp32 or fp16+TwoSum), arrival rate set so
    that the offered work is about 80% of the measured solo throughput;
    admission by device footprint (budget: 80% of free HBM unless given);
    continuous batching in chunks of `chunk` steps, each kernel group on its
    own stream.  A request's inputs are drawn when it is admitted.
    glups: solo rates by (kind, precision)."""
    import workloads
    from paper_2310_00236_amd import serve

    def solo(r):
        return glups[(r.kind, r.precision)] * 1e9

    def cells(r):
        return r.size ** 2 if r.kind == "acoustic2d" else r.size ** 3

    probe = workloads.request_stream(nreq, rate=1.0, seed=seed)
    mean_work = sum(cells(r) * r.nsteps / solo(r) for r in probe) / len(probe)
    rate = 0.8 / mean_work
    reqs = workloads.request_stream(nreq, rate=rate, seed=seed)

    def problem(r, dt=1.0, dx=1.0):
        storage, comp = ("f32", "none") if r.precision == "f32" else ("f16", "twosum")
        if r.kind == "acoustic2d":
            return hw.Problem("acoustic2d", r.size, r.size, 1, 4, storage, comp, dx, dt, 0, 0)
        return hw.Problem("elastic3d", r.size, r.size, r.size, 2, storage, comp, dx, dt, 0, 0)

    def inputs(r):
        w = workloads.request_problem(r)
        mat = [w.rho, w.kappa] if r.kind == "acoustic2d" else [w.rho, w.lam, w.mu]
        return problem(r, w.dt, w.dx), mat, w.fields()

    jobs = []
    for r in reqs:
        pb = problem(r)               # the footprint does not depend on dt
        jobs.append(serve.Job(id=r.index, arrival=r.arrival, footprint=hw.footprint(pb),
                              nsteps=r.nsteps, cells=pb.cells,
                              payload=(lambda r=r: inputs(r))))
    if budget is None:
        free, _ = torch.cuda.mem_get_info()
        budget = int(0.8 * free)
    def note(j):
        print(f"# served request {j.id} ({len(jobs)} in the stream): latency "
              f"{j.latency:.2f} s", file=sys.stderr, flush=True)
        # the result reached the host (the latency counts that); the
        # benchmark keeps none of them (a 384^3 request's fields and
        # compensation terms are 8 GB of fp64)
        j.result = None

    summary, done = serve.serve(jobs, budget, chunk_steps=chunk, on_retire=note)
    # the fraction of the wall time the GPU would need to run the served work
    # one request at a time at the solo rates
    busy = sum(cells(r) * r.nsteps / solo(r) for r in reqs
               if any(j.id == r.index for j in done))
    summary.update({"requests": nreq, "arrival_rate_per_s": rate,
                    "hbm_budget_bytes": budget, "chunk_steps": chunk,
                    "utilisation_at_solo_rates": busy / summary["wall_s"],
                    "workload": "Poisson stream, 70% 2D order-4 512^2-4096^2 / 30% 3D "
                                "128^3-384^3, 1000-10000 steps, fp32 or fp16+TwoSum"})
    print(f"# serving (budget {budget / 1e9:.1f} GB): {summary}", file=sys.stderr, flush=True)
    return summary


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile shape index (-1: best from the tuning table)")
    ap.add_argument("--variants", default="all",
                    help="comma list of storage+comp, e.g. f16+twosum,f32+none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--elastic-n", type=int, default=512)
    ap.add_argument("--elastic-steps", type=int, default=2000)
    ap.add_argument("--shots", type=int, default=64)
    ap.add_argument("--requests", type=int, default=120,
                    help="requests of the serving stream (80%% of free HBM as budget)")
    ap.add_argument("--small-budget-requests", type=int, default=40,
                    help="requests of the second serving stream, under an 8 GB budget")
    ap.add_argument("--drift-steps", type=int, default=10000,
                    help="length of each variant's untimed full run, for the energy "
                         "drift against the FP64 oracle (0: skip)")
    ap.add_argument("--sections", default="2d,3d,batched,serving,paper,app_a",
                    help="comma list of workloads to run: 2d (always reported), "
                         "3d, batched, serving, paper (the Sec. 3 experiment), "
                         "app_a (the elastic experiment of App. A)")
    ap.add_argument("--paper-steps", type=int, default=60000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates "
                         "the HBM byte counters against a known size)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "repeats": 6,
                          "read_plus_write_gbs": 2 * a.numel() * 4 / ms / 1e6}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2310_00236_amd as hw
    import workloads
    from paper_2310_00236_amd import tuning

    torch.cuda.init()
    w = workloads.layered2d(args.n, nsteps=args.steps)
    variants = VARIANTS if args.variants == "all" else \
        [tuple(v.split("+")) for v in args.variants.split(",")]
    results = {}
    tiles = {}
    for storage, comp in variants:
        tile = args.tile if args.tile >= 0 else tuning.best_tile(
            "acoustic2d", w.order, storage, comp, w.nx, w.ny)
        tiles[f"{storage}+{comp}"] = tile
        results[f"{storage}+{comp}"] = run_variant(hw, torch, w, storage, comp,
                                                   args.steps, args.warmup, tile)
        print(f"# {storage}+{comp}: {results[f'{storage}+{comp}']}", file=sys.stderr,
              flush=True)
    head_key = "f16+twosum" if "f16+twosum" in results else next(iter(results))
    head = results[head_key]
    cells = w.nx * w.ny
    # the full run of every variant (untimed), energy against the FP64 oracle
    if args.drift_steps > 0:
        gold = read_layered_golden() if (w.nx, w.ny) == (4096, 4096) else {}
        for key, r in results.items():
            storage, comp = key.split("+")
            r["full_run"] = drift_run(hw, w, storage, comp, tiles[key], args.drift_steps,
                                      gold.get(storage))
            print(f"# {key} full run: {r['full_run']}", file=sys.stderr, flush=True)
    traffic = measured_traffic(head_key)
    shape = hw.tiles("acoustic2d")[tiles[head_key]]
    per = head["steps_per_launch"]
    storage, comp = head_key.split("+")
    roofline = {
        "bound": "hbm",
        "achieved": head["hbm_gbs_algorithmic"],
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": head["hbm_gbs_algorithmic"] / PEAK_HBM_GBS,
        "traffic": traffic,
        "kernel": {1: "ac2d_march1_kernel", 4: "ac2d_step2_1_kernel",
                   5: "ac2d_step2_1_kernel"}.get(shape[3], "ac2d_step1_kernel"),
        "tile": hw.tile_label(shape),
        "steps_per_launch": per,
        "bytes_per_cell_launch": bytes_per_cell(storage, comp),
        "bytes_per_cell_step": head["bytes_per_cell"],
        "cells_per_launch": cells,
        "launch_ms": head["kernel_ms"] * per,
        "kernel_ms": head["kernel_ms"],
        # the throughput against the HBM roofline of a kernel that reads and
        # writes the state every step (32 B per cell-step for fp16 +
        # compensation and for fp32: 250 GLUPS at 8 TB/s)
        "frac_of_one_step_roofline": head["glups"] * bytes_per_cell(storage, comp)
        / PEAK_HBM_GBS,
    }
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    extra = {}
    sections = set(args.sections.split(","))
    if "3d" in sections or "serving" in sections:
        extra["elastic3d"] = run_elastic(hw, torch, args.elastic_n, args.elastic_steps,
                                         20, [("f16", "twosum"), ("f32", "none")])
    if "batched" in sections:
        extra["batched"] = run_batched(hw, torch, args.shots)
    if "serving" in sections:
        e3 = extra["elastic3d"]["variants"]
        solo = {("acoustic2d", "f16+comp"): results.get("f16+twosum", head)["glups"],
                ("acoustic2d", "f32"): results.get("f32+none", head)["glups"],
                ("elastic3d", "f16+comp"): e3["f16+twosum"]["glups"],
                ("elastic3d", "f32"): e3["f32+none"]["glups"]}
        extra["serving"] = run_serving(hw, torch, args.requests, solo)
        if args.small_budget_requests > 0:
            extra["serving_8GB"] = run_serving(hw, torch, args.small_budget_requests, solo,
                                               budget=8 * 10 ** 9, seed=workloads.seed_for(5, 9999))
    if "paper" in sections:
        extra["paper2d"] = run_paper(hw, torch, args.paper_steps)
    if "app_a" in sections:
        extra["elastic2d_app_a"] = run_app_a(hw, torch, args.paper_steps)
    f32 = results.get("f32+none")
    out = {
        "metric": METRIC,
        "value": head["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if head_key.startswith("f16") else head_key.split("+")[0],
        "data": "synthetic",
        "config": {"workload": f"acoustic2d order-4 {w.nx}x{w.ny} periodic, "
                               f"4-layer medium, CFL 0.4, 4 Gaussian pulses, "
                               f"{args.steps} steps",
                   "variant": head_key, "tile": list(hw.tiles("acoustic2d")[tiles[head_key]]),
                   "energy_every": ENERGY_EVERY},
        "energy_drift": head["energy_drift_window"],
        "energy_drift_vs_fp64": head.get("full_run", {}).get("energy_drift_vs_fp64"),
        "energy_drift_steps": head.get("full_run", {}).get("steps"),
        "vs_f32": (head["glups"] / f32["glups"]) if f32 else None,
        "variants": {k: {"glups": v["glups"], "ms_per_step": v["ms_per_step"],
                         "steps_per_launch": v["steps_per_launch"],
                         "energy_drift_window": v["energy_drift_window"],
                         "energy_drift_vs_fp64": v.get("full_run", {}).get(
                             "energy_drift_vs_fp64"),
                         "full_run": v.get("full_run"),
                         "kernel_ms": v["kernel_ms"],
                         "hbm_gbs_algorithmic": v["hbm_gbs_algorithmic"],
                         "frac_hbm": v["hbm_gbs_algorithmic"] / PEAK_HBM_GBS,
                         "tile": list(hw.tiles("acoustic2d")[tiles[k]])}
                     for k, v in results.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    if "serving" in extra:
        out["p50_latency_s"] = extra["serving"]["p50_latency_s"]
        out["p99_latency_s"] = extra["serving"]["p99_latency_s"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
