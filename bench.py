"""Benchmark of the Hilbert-ordered SEM time step on one MI355X.

Headline (``value``): GDOF*steps/s of the FP32 single-shot step on the layered jittered
1024 x 1024-element p=4 mesh (16.8 M global nodes), Hilbert element order, inputs resident
in HBM. One "step" = one fused launch doing the whole hot path: gather, tensor-product
stiffness, scatter-add, diagonal-mass-inverse leapfrog update, source and receivers.

Extra legs on the same JSON line: the FP64 step on the same mesh, the 64-shot FP32 batch
and single-shot FP64 step on the 512 x 512 mesh, the adjoint-gradient cost ratio on the
8-shot inversion workload, and the element-order sweep. The ``cpu_baseline`` leg times the
FP64 CPU oracle on a bounded section of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--legs main,fp64,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ALL_LEGS = ("main", "fp64", "batch", "adjoint", "orders", "cpu")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sim(sem, wl, precision, order="hilbert", n_shots=None, **kw):
    t0 = time.perf_counter()
    s = sem.Simulator(wl.vxy, wl.quads, wl.c2, wl.p, precision=precision, order=order,
                      n_shots=n_shots or wl.n_shots, **kw)
    s.set_sources(wl.src_xy, wl.src_shot, wl.f0)
    s.set_receivers(wl.rec_xy)
    return s, time.perf_counter() - t0


def time_steps(torch, sim, steps, warmup, record=True):
    """Average time of one step over ``steps`` launches, HIP events on the sim's stream."""
    sim.reset()
    sim.run(warmup, record=False)
    traces = None
    if record and sim.n_receivers:
        traces = torch.empty((sim.n_shots, sim.n_receivers, steps), dtype=sim.torch_dtype, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.run(steps, traces=traces, record=record)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    return ms / 1e3 / steps, traces


def leg_summary(sim, sec_per_step, label):
    inf = sim.info()
    gdof = inf["n_nodes"] * inf["n_shots"] / sec_per_step / 1e9
    gbs = inf["alg_bytes_per_step"] / sec_per_step / 1e9
    return {
        "label": label,
        "gdof_steps_per_s": gdof,
        "us_per_step": sec_per_step * 1e6,
        "alg_bytes_per_step": inf["alg_bytes_per_step"],
        "achieved_GBs": gbs,
        "hbm_frac": gbs / HBM_PEAK_GBS,
        "n_nodes": inf["n_nodes"],
        "n_elements": inf["n_elements"],
        "n_shots": inf["n_shots"],
        "tile_elems": inf["tile_elems"],
        "shot_lanes": inf["shot_lanes"],
        "halo_ratio": inf["halo_elements"] / inf["n_elements"],
        "setup_s": inf["setup_seconds"],
        "reorder_s": inf["reorder_seconds"],
    }


def cpu_baseline(n=256, steps=200):
    """FP64 CPU oracle on an n x n-element section of the layered jittered p=4 workload."""
    import workloads
    from oracle import solver
    wl = workloads.workload("layered1024", n=n)
    t0 = time.perf_counter()
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    t_setup = time.perf_counter() - t0
    dt = o.dt_cfl()
    src = solver.snap_to_nodes(wl.src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    o.run(2, dt, src, [0], wl.f0, rec_nodes=rec)
    t0 = time.perf_counter()
    o.run(steps, dt, src, [0], wl.f0, rec_nodes=rec)
    t = time.perf_counter() - t0
    return {
        "value": o.n_nodes * steps / t / 1e9,
        "unit": "GDOF*steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"FP64 oracle (scipy CSR stiffness, numpy update), {n}x{n}-element section of "
                   f"the layered jittered p=4 workload ({o.n_nodes} nodes), {steps} steps after "
                   f"2 warm-up steps; operator assembly ({t_setup:.1f} s) excluded"),
        "sec_per_step": t / steps,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--legs", default=",".join(ALL_LEGS))
    ap.add_argument("--quick", action="store_true", help="headline leg only")
    ap.add_argument("--n", type=int, default=None, help="elements per side of the headline mesh")
    ap.add_argument("--order", default="hilbert", choices=["hilbert", "morton", "lex", "random"],
                    help="element order of the headline leg")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"], help="headline precision")
    ap.add_argument("--workload", default="layered1024", choices=["layered1024", "graded1414", "batch512"],
                    help="headline workload (default: the layered 1024^2 p=4 mesh)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU sharding is a "
              "design note, not part of this build.", file=sys.stderr)
        sys.exit(2)
    legs = ("main",) if args.quick else tuple(x for x in args.legs.split(",") if x)

    import torch
    import workloads
    from paper_2104_08416_amd import sem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    out = {}
    if args.copy_calib:
        # plain copy of 2^28 floats (1 GiB read + 1 GiB written per launch), timed
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3 / 5
        out["copy_calib"] = {"bytes_per_launch": 2 * 4 * (1 << 28), "GBs": 2 * 4 * (1 << 28) / sec / 1e9}
        del src, dst
    # ---------------------------------------------------------------- headline
    wl = workloads.workload(args.workload, n=args.n)
    label = f"{args.workload} n={wl.nx} p={wl.p} {args.precision} {args.order} S={wl.n_shots}"
    log(f"[bench] headline: {label}, setup ...")
    sim, t_setup = make_sim(sem, wl, args.precision, args.order)
    log(f"[bench] setup {t_setup:.1f} s, timing {args.steps} steps")
    sps, _ = time_steps(torch, sim, args.steps, args.warmup)
    main_leg = leg_summary(sim, sps, label)
    log(f"[bench] headline {main_leg['gdof_steps_per_s']:.1f} GDOF*steps/s, {main_leg['us_per_step']:.1f} us/step")
    sim.close()

    if "fp64" in legs:
        log("[bench] fp64 leg")
        s64, _ = make_sim(sem, wl, "f64", "hilbert")
        sps64, _ = time_steps(torch, s64, min(args.steps, 300), args.warmup)
        out["fp64"] = leg_summary(s64, sps64, "layered1024 p4 f64 hilbert S=1")
        s64.close()
    if "orders" in legs:
        out["orders"] = {"hilbert": {k: main_leg[k] for k in ("gdof_steps_per_s", "hbm_frac", "halo_ratio",
                                                              "setup_s", "reorder_s")}}
        for order in ("morton", "lex", "random"):
            log(f"[bench] order {order}")
            so, _ = make_sim(sem, wl, "f32", order)
            spo, _ = time_steps(torch, so, min(args.steps, 200), 5)
            lg = leg_summary(so, spo, order)
            out["orders"][order] = {k: lg[k] for k in ("gdof_steps_per_s", "hbm_frac", "halo_ratio",
                                                       "setup_s", "reorder_s")}
            so.close()
    if "batch" in legs:
        log("[bench] batch leg: 512^2 p=4, 64 shots FP32 vs single-shot FP64")
        wb = workloads.workload("batch512")
        sb, _ = make_sim(sem, wb, "f32", "hilbert")
        spb, _ = time_steps(torch, sb, min(args.steps, 200), 10)
        out["batch64"] = leg_summary(sb, spb, "batch512 p4 f32 hilbert S=64")
        sb.close()
        w1 = workloads.workload("batch512", n_shots=1)
        s1, _ = make_sim(sem, w1, "f64", "hilbert")
        sp1, _ = time_steps(torch, s1, min(args.steps, 300), 10)
        out["batch64"]["single_shot_f64"] = leg_summary(s1, sp1, "batch512 p4 f64 hilbert S=1")
        out["batch64"]["speedup_vs_single_shot_f64"] = (
            out["batch64"]["gdof_steps_per_s"] / out["batch64"]["single_shot_f64"]["gdof_steps_per_s"])
        s1.close()
    if "adjoint" in legs:
        log("[bench] adjoint leg: 512^2 p=4, 8 shots, 1500 steps, checkpoints every 40")
        wa = workloads.workload("adjoint512")
        sa, _ = make_sim(sem, wa, "f32", "hilbert")
        n = wa.nsteps
        sa.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = sa.run(n)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        res = (tr * 0.5).contiguous()
        t0 = time.perf_counter()
        g = sa.adjoint_gradient(res, n, wa.ckpt_every)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        out["adjoint"] = {"forward_s": t_fwd, "gradient_s": t_adj, "cost_ratio": t_adj / t_fwd,
                          "steps": n, "ckpt_every": wa.ckpt_every, "n_shots": wa.n_shots,
                          "grad_finite": bool(torch.isfinite(g).all().item())}
        sa.close()
    cpu = None
    if "cpu" in legs:
        log("[bench] cpu_baseline leg (oracle)")
        cpu = cpu_baseline()

    line = {
        "metric": "SEM GDOF*steps/s (FP32 single-shot, Hilbert order); FP64, 64-shot batch, "
                  "adjoint cost and % HBM as extra fields",
        "value": main_leg["gdof_steps_per_s"],
        "unit": "GDOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["us_per_step"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": (f"layered jittered {wl.nx}x{wl.nx} quads, p=4, six layers 1500-4500 m/s "
                                f"+-5%, Ricker 15 Hz at centre, 128 receivers, {args.order} order, 1 shot")
                   if args.workload == "layered1024" else label,
                   "n_nodes": main_leg["n_nodes"], "n_elements": main_leg["n_elements"],
                   "tile_elems": main_leg["tile_elems"], "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": main_leg["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_leg["hbm_frac"], "traffic": None},
        "cpu_baseline": cpu,
        "main": main_leg,
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
