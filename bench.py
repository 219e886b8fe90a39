"""Benchmark of the Hilbert-ordered SEM time step on one MI355X.

Headline (``value``): GDOF*steps/s of the FP32 single-shot step on the layered jittered
1024 x 1024-element p=4 mesh (16.8 M global nodes), Hilbert element order, inputs resident
in HBM. One "step" = one fused launch doing the whole hot path: gather, tensor-product
stiffness, scatter-add, diagonal-mass-inverse leapfrog update, source and receivers.

Extra legs on the same JSON line: the FP64 step on the same mesh, the 64-shot FP32 batch
and single-shot FP64 step on the 512 x 512 mesh, the adjoint-gradient cost ratio on the
8-shot inversion workload, the element-order sweep, and the graded 1414 x 1414 p=5 mesh
in Hilbert, Morton and random order. The ``cpu_baseline`` leg times the
FP64 CPU oracle on a bounded section of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--legs main,fp64,...]
       python bench.py --profile-summary DIR --steps K --kernel NAME   (no GPU: turns the
           rocprofv3 CSV output under DIR into the markdown summaries kept in profiles/)

Roofline fields: ``achieved`` = algorithmic bytes of one step (per element nq int32 ids,
3 nq geometric factors and c2; per node dt/M and u, v read and written) / the average
step-kernel duration from HIP events on the kernel's stream. ``traffic`` = FETCH_SIZE +
WRITE_SIZE bytes per step-kernel dispatch from rocprofv3 counter runs, each scaled by the
ratio of bytes a plain 1 GiB device copy moves to what the same counter reads for it; it
is read from the headline summary in profiles/ and is null when the kernel sources have
changed since those counters were taken.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
ALL_LEGS = ("main", "fp64", "scatter", "heun", "tri", "batch", "adjoint", "orders", "graded", "shard", "cpu")
CHUNKS = 5                     # the timed steps are event-timed in this many chunks (median)
KERNEL_SOURCES = ("kernels.hip", "kernels.h", "api.hip", "plan.cpp", "plan.h")
HEADLINE_PROFILE = os.path.join(ROOT, "profiles", "step_rows_kernel_layered1024_f32_hilbert.md")
COPY_BYTES = 1 << 30           # the calibration copy reads and writes 1 GiB each


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
    """Time ``steps`` launches after ``warmup`` untimed ones, with HIP events on the sim's
    stream around the whole run and around each of CHUNKS equal chunks of it. Returns the
    mean time per step over the whole run, the traces, and the median of the chunk means."""
    sim.reset()
    sim.run(warmup, record=False)
    traces = None
    if record and sim.n_receivers:
        traces = torch.empty((sim.n_shots, sim.n_receivers, steps), dtype=sim.torch_dtype, device="cuda")
    chunks = max(1, min(CHUNKS, steps))
    bounds = [steps * k // chunks for k in range(chunks + 1)]
    # one trace buffer per chunk, allocated before the timed region
    parts = [torch.empty((sim.n_shots, sim.n_receivers, bounds[k + 1] - bounds[k]), dtype=sim.torch_dtype,
                         device="cuda") if traces is not None else None for k in range(chunks)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(chunks + 1)]
    evs[0].record(stream)
    for k in range(chunks):
        sim.run(bounds[k + 1] - bounds[k], traces=parts[k], record=record)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    if traces is not None:
        torch.cat(parts, dim=2, out=traces)
    total = evs[0].elapsed_time(evs[-1]) / 1e3 / steps
    per = sorted(evs[k].elapsed_time(evs[k + 1]) / 1e3 / (bounds[k + 1] - bounds[k]) for k in range(chunks))
    return total, traces, per[len(per) // 2]


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
        "kernel_bytes_per_step": inf["kernel_bytes_per_step"],
        "kernel_bytes_GBs": inf["kernel_bytes_per_step"] / sec_per_step / 1e9,
        "block_threads": inf["block_threads"],
        "n_nodes": inf["n_nodes"],
        "n_elements": inf["n_elements"],
        "n_shots": inf["n_shots"],
        "tile_elems": inf["tile_elems"],
        "shot_lanes": inf["shot_lanes"],
        "halo_ratio": inf["halo_elements"] / inf["n_elements"],
        "setup_s": inf["setup_seconds"],
        "reorder_s": inf["reorder_seconds"],
        "n_colours": inf["n_colours"],
    }


def sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_08416_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_record(path):
    """The JSON block of a profile summary, or None."""
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    return json.loads(m.group(1)) if m else None


def headline_traffic():
    """FETCH + WRITE bytes per step-kernel dispatch of the headline, if the summary in
    profiles/ was taken with the current kernel sources."""
    rec = profile_record(HEADLINE_PROFILE)
    if rec is None or rec.get("sources_sha256") != sources_sha256():
        return None
    return rec["traffic_bytes_per_dispatch"]


def _rows(d, pattern):
    fs = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not fs:
        raise SystemExit(f"no {pattern} under {d}")
    with open(fs[0]) as fh:
        return list(csv.DictReader(fh))


def _counter(d, name, kernel, last):
    vals = [float(r["Counter_Value"]) for r in _rows(d, "*counter_collection.csv")
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == name]
    vals = vals[-last:]
    return sum(vals) / len(vals)


def _copy_counter(d, name):
    rows = [r for r in _rows(d, "*counter_collection.csv")
            if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name]
    top = max(int(r["Grid_Size"]) for r in rows)
    vals = [float(r["Counter_Value"]) for r in rows if int(r["Grid_Size"]) == top]
    return sum(vals) / len(vals)


def profile_summary(d, kernel, steps, counter_steps, per_step=1):
    """Markdown summary of rocprofv3 runs under d: trace/ (kernel trace + stats) and, if
    present, fetch/, write/ (FETCH_SIZE, WRITE_SIZE with the copy calibration) and tcc/
    (TCC_HIT_sum, TCC_MISS_sum). Averages use the last ``steps`` steps of ``kernel`` in the
    trace and the last ``counter_steps`` in the counter runs (the timed steps); a step
    launches ``kernel`` ``per_step`` times (one launch per colour for the colour scatter),
    and the figures are per dispatch."""
    out = []
    steps *= per_step
    counter_steps *= per_step
    stats = _rows(os.path.join(d, "trace"), "*kernel_stats.csv")
    trace = [r for r in _rows(os.path.join(d, "trace"), "*kernel_trace.csv") if kernel in r["Kernel_Name"]]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace][-steps:]
    avg_us = sum(durs) / len(durs)
    out.append("| kernel | calls | avg us | total % |")
    out.append("|---|---|---|---|")
    for r in stats[:8]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f} |")
    out.append("")
    out.append(f"`{kernel}`: last {len(durs)} dispatches (the timed steps) average {avg_us:.1f} us, "
               f"min {min(durs):.1f}, max {max(durs):.1f}.")
    if per_step > 1:
        out.append(f"{per_step} dispatches per step: {avg_us * per_step:.1f} us of `{kernel}` per step.")
    rec = {"kernel": kernel, "dispatches": len(durs), "avg_us": avg_us, "dispatches_per_step": per_step,
           "sources_sha256": sources_sha256()}
    if os.path.isdir(os.path.join(d, "fetch")) and os.path.isdir(os.path.join(d, "write")):
        f_kib = _counter(os.path.join(d, "fetch"), "FETCH_SIZE", kernel, counter_steps)
        w_kib = _counter(os.path.join(d, "write"), "WRITE_SIZE", kernel, counter_steps)
        cf = _copy_counter(os.path.join(d, "fetch"), "FETCH_SIZE")
        cw = _copy_counter(os.path.join(d, "write"), "WRITE_SIZE")
        fs, ws = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
        fb, wb = f_kib * 1024 * fs, w_kib * 1024 * ws
        out.append("")
        out.append(f"Copy calibration (1 GiB read + 1 GiB written): FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE "
                   f"{cw:.0f} KiB per dispatch, so scale factors {fs:.3f} (fetch) and {ws:.3f} (write).")
        out.append(f"`{kernel}` per dispatch: FETCH_SIZE {f_kib:.0f} KiB -> {fb / 1e6:.1f} MB, WRITE_SIZE "
                   f"{w_kib:.0f} KiB -> {wb / 1e6:.1f} MB, traffic {(fb + wb) / 1e6:.1f} MB.")
        rec.update({"fetch_kib": f_kib, "write_kib": w_kib, "fetch_scale": fs, "write_scale": ws,
                    "fetch_bytes_per_dispatch": fb, "write_bytes_per_dispatch": wb,
                    "traffic_bytes_per_dispatch": fb + wb})
    if os.path.isdir(os.path.join(d, "tcc")):
        h = _counter(os.path.join(d, "tcc"), "TCC_HIT_sum", kernel, counter_steps)
        m = _counter(os.path.join(d, "tcc"), "TCC_MISS_sum", kernel, counter_steps)
        out.append(f"L2 (TCC) hit rate {h / (h + m):.3f} ({h:.0f} hits, {m:.0f} misses per dispatch).")
        rec.update({"l2_hit": h / (h + m)})
    # other counter passes (pmc*/): every counter of the kernel, averaged per dispatch
    pmc = {}
    for sub in sorted(g for g in glob.glob(os.path.join(d, "pmc*")) if os.path.isdir(g)):
        rows = [r for r in _rows(sub, "*counter_collection.csv") if kernel in r["Kernel_Name"]]
        for name in sorted({r["Counter_Name"] for r in rows}):
            vals = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == name][-counter_steps:]
            pmc[name] = sum(vals) / len(vals)
    if pmc:
        out.append("")
        out.append("| counter (per dispatch) | value |")
        out.append("|---|---|")
        for name, v in pmc.items():
            out.append(f"| {name} | {v:.4g} |")
        ratios = {}
        wc = pmc.get("SQ_WAVE_CYCLES")
        if wc:
            for name, label in (("SQ_ACTIVE_INST_VALU", "VALU issue per wave-cycle"),
                                ("SQ_ACTIVE_INST_LDS", "LDS issue per wave-cycle"),
                                ("SQ_ACTIVE_INST_VMEM", "VMEM issue per wave-cycle"),
                                ("SQ_WAIT_INST_ANY", "waiting on s_waitcnt per wave-cycle"),
                                ("SQ_WAIT_ANY", "waiting (any) per wave-cycle")):
                if name in pmc:
                    ratios[label] = pmc[name] / wc
        if "SQ_LDS_BANK_CONFLICT" in pmc and pmc.get("SQ_ACTIVE_INST_LDS"):
            ratios["LDS bank-conflict cycles per LDS-active cycle"] = pmc["SQ_LDS_BANK_CONFLICT"] / pmc["SQ_ACTIVE_INST_LDS"]
        if wc and pmc.get("SQ_BUSY_CYCLES"):
            ratios["resident waves per busy SQ cycle (all CUs of an SE)"] = wc / pmc["SQ_BUSY_CYCLES"]
        for k, v in ratios.items():
            out.append(f"- {k}: {v:.3f}")
        rec.update({"pmc": pmc, "pmc_ratios": ratios})
    for log_name in ("trace.log", "fetch.log"):
        lp = os.path.join(d, log_name)
        if os.path.exists(lp):
            for line in open(lp):
                if line.startswith("{"):
                    b = json.loads(line)
                    rec.setdefault("bench_us_per_step", b["main"]["us_per_step"])
                    rec.setdefault("alg_bytes_per_step", b["main"]["alg_bytes_per_step"])
                    out.append(f"bench.py in the `{log_name[:-4]}` run: {b['main']['us_per_step']:.1f} us/step "
                               f"(HIP events), {b['main']['alg_bytes_per_step'] / 1e6:.1f} MB algorithmic.")
                    break
    out.append("")
    out.append("```json")
    out.append(json.dumps(rec, indent=1))
    out.append("```")
    return "\n".join(out)


def _oracle_section(n):
    import workloads
    from oracle import solver
    wl = workloads.workload("layered1024", n=n)
    t0 = time.perf_counter()
    o = solver.SEM(wl.vxy, wl.quads, wl.c2, wl.p)
    t_setup = time.perf_counter() - t0
    dt = o.dt_cfl()
    src = solver.snap_to_nodes(wl.src_xy, o.node_xy)
    rec = solver.snap_to_nodes(wl.rec_xy, o.node_xy)
    return wl, o, dt, src, rec, t_setup


def _oracle_worker(args):
    """One process of the all-core oracle run: its own copy of the section, timed steps."""
    n, steps = args
    wl, o, dt, src, rec, _ = _oracle_section(n)
    o.run(2, dt, src, [0], wl.f0, rec_nodes=rec)
    t0 = time.perf_counter()
    o.run(steps, dt, src, [0], wl.f0, rec_nodes=rec)
    return o.n_nodes, steps, time.perf_counter() - t0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n=256, steps=1000, all_core_steps=200):
    """FP64 CPU oracle on an n x n-element section of the layered jittered p=4 workload: one
    process on one core, then one process per core (up to 16, the host share of one GPU)
    each stepping its own copy of the section (the oracle itself is single-threaded)."""
    import multiprocessing as mp
    wl, o, dt, src, rec, t_setup = _oracle_section(n)
    o.run(2, dt, src, [0], wl.f0, rec_nodes=rec)
    t0 = time.perf_counter()
    o.run(steps, dt, src, [0], wl.f0, rec_nodes=rec)
    t = time.perf_counter() - t0
    nodes = o.n_nodes
    del o
    cores = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(n, all_core_steps)] * cores)
    all_rate = sum(nn * st / sec for nn, st, sec in res) / 1e9
    return {
        "value": nodes * steps / t / 1e9,
        "unit": "GDOF*steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"FP64 oracle (scipy CSR stiffness, numpy update), {n}x{n}-element section of "
                   f"the layered jittered p=4 workload ({nodes} nodes), {steps} steps after "
                   f"2 warm-up steps; operator assembly ({t_setup:.1f} s) excluded"),
        "sec_per_step": t / steps,
        "cpu_model": cpu_model(),
        "all_cores": {"value": all_rate, "cores": cores,
                      "sample": f"{cores} processes, each its own copy of the same section, "
                                f"{all_core_steps} steps each, aggregate node-steps/s"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--legs", default=",".join(ALL_LEGS))
    ap.add_argument("--quick", action="store_true", help="headline leg only")
    ap.add_argument("--n", type=int, default=None, help="elements per side of the headline mesh")
    ap.add_argument("--order", default="hilbert",
                    choices=["hilbert", "morton", "lex", "random", "connectivity", "distance"],
                    help="element order of the headline leg")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"], help="headline precision")
    ap.add_argument("--workload", default="layered1024",
                    choices=["layered1024", "graded1414", "batch512", "tri2000"],
                    help="headline workload (default: the layered 1024^2 p=4 mesh)")
    ap.add_argument("--formulation", default="leapfrog", choices=["leapfrog", "heun"],
                    help="headline formulation: second-order leapfrog or the first-order system with Heun")
    ap.add_argument("--scatter", default="auto", choices=["auto", "lds_atomic", "colour", "atomic"],
                    help="headline scatter: owner-tile LDS (auto), colour passes or global atomics")
    ap.add_argument("--copy-calib", action="store_true",
                    help="headline leg only, as in the counter runs (the 1 GiB copy always runs first)")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="summarise rocprofv3 CSV output under DIR (no GPU) and exit")
    ap.add_argument("--kernel", default="step_rows_kernel", help="kernel of --profile-summary")
    ap.add_argument("--counter-steps", type=int, default=10,
                    help="--steps of the counter runs summarised by --profile-summary")
    ap.add_argument("--per-step", type=int, default=1,
                    help="--profile-summary: launches of --kernel per step")
    args = ap.parse_args()
    if args.profile_summary:
        print(profile_summary(args.profile_summary, args.kernel, args.steps, args.counter_steps, args.per_step))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path; the `shard` leg measures one GPU's share of an 8-way split.", file=sys.stderr)
        sys.exit(2)
    legs = ("main",) if (args.quick or args.copy_calib) else tuple(x for x in args.legs.split(",") if x)

    cpu = None
    if "cpu" in legs:
        # first, so that its worker processes fork before this process touches the GPU
        log("[bench] cpu_baseline leg (oracle, one core then all cores)")
        cpu = cpu_baseline()

    import torch
    import workloads
    from paper_2104_08416_amd import sem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    out = {}
    # plain device copy of 2^28 floats (1 GiB read + 1 GiB written per launch): the HBM rate
    # a streaming kernel reaches on this device, and the reference of the counter scaling
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
    copy_gbs = 2 * 4 * (1 << 28) / sec / 1e9
    out["copy_calib"] = {"bytes_per_launch": 2 * 4 * (1 << 28), "GBs": copy_gbs}
    del src, dst
    # ---------------------------------------------------------------- headline
    wl = workloads.workload(args.workload, n=args.n)
    label = f"{args.workload} n={wl.nx} p={wl.p} {args.precision} {args.order} S={wl.n_shots}"
    if args.formulation != "leapfrog":
        label += f" {args.formulation}"
    if args.scatter != "auto":
        label += f" scatter={args.scatter}"
    log(f"[bench] headline: {label}, setup ...")
    sim, t_setup = make_sim(sem, wl, args.precision, args.order, formulation=args.formulation,
                            scatter=args.scatter)
    log(f"[bench] setup {t_setup:.1f} s, timing {args.steps} steps")
    sps, _, sps_med = time_steps(torch, sim, args.steps, args.warmup)
    main_leg = leg_summary(sim, sps, label)
    main_leg["median_chunk_us_per_step"] = sps_med * 1e6
    log(f"[bench] headline {main_leg['gdof_steps_per_s']:.1f} GDOF*steps/s, {main_leg['us_per_step']:.1f} us/step")
    elem_new2old, _ = sim.permutations()
    main_dt = sim.dt
    sim.close()

    if "shard" in legs and args.workload == "layered1024" and wl.quads.shape[1] == 4:
        # One GPU's share of an 8-way split of the single-shot step (each GPU takes a
        # contiguous eighth of the curve's element order): that eighth as a mesh of its own, at
        # its real shape, and the interface an 8-way split would exchange per step (no
        # exchange is run: the library has no multi-GPU path)
        G = 8
        ne = wl.quads.shape[0]
        log(f"[bench] shard leg: the first 1/{G} of the Hilbert element order as one GPU's share")
        chunk = np.sort(elem_new2old[: ne // G])
        verts, inv = np.unique(wl.quads[chunk].ravel(), return_inverse=True)
        sq = inv.reshape(-1, 4).astype(np.int32)
        ss = sem.Simulator(wl.vxy[verts], sq, wl.c2[chunk], wl.p, precision="f32", order="hilbert", dt=main_dt)
        ssps, _, _ = time_steps(torch, ss, min(args.steps, 300), args.warmup, record=False)
        lg = leg_summary(ss, ssps, f"layered1024 p4 f32 hilbert S=1, elements [0, E/{G}) of the curve")
        ss.close()
        inside = np.zeros(ne, bool)
        inside[chunk] = True
        shared_v = np.intersect1d(np.unique(wl.quads[inside]), np.unique(wl.quads[~inside]))

        def edges(q):
            e = np.stack([q, np.roll(q, -1, axis=1)], axis=2).reshape(-1, 2)
            e.sort(axis=1)
            return np.unique(e[:, 0].astype(np.int64) * wl.vxy.shape[0] + e[:, 1])

        shared_e = np.intersect1d(edges(wl.quads[inside]), edges(wl.quads[~inside]))
        iface = int(shared_v.size + (wl.p - 1) * shared_e.size)
        out["shard"] = {k: lg[k] for k in ("label", "gdof_steps_per_s", "us_per_step", "hbm_frac", "n_nodes",
                                             "n_elements", "halo_ratio")}
        out["shard"].update({"gpus_in_split": G, "rate_vs_whole_mesh": lg["gdof_steps_per_s"] /
                             main_leg["gdof_steps_per_s"], "interface_nodes": iface,
                             "interface_bytes_fp32": 4 * iface})

    if "fp64" in legs:
        log("[bench] fp64 leg")
        s64, _ = make_sim(sem, wl, "f64", "hilbert")
        sps64, _, _ = time_steps(torch, s64, min(args.steps, 300), args.warmup)
        out["fp64"] = leg_summary(s64, sps64, "layered1024 p4 f64 hilbert S=1")
        s64.close()
    if "scatter" in legs:
        # the paper's colouring (one launch per colour, plain read-modify-write of a global r,
        # then a node pass) and global atomics, against the owner-tile LDS scatter
        out["scatter"] = {"lds_atomic": {"us_per_step": main_leg["us_per_step"],
                                         "gdof_steps_per_s": main_leg["gdof_steps_per_s"]}}
        for sc in ("colour", "atomic"):
            log(f"[bench] scatter {sc}")
            sc_sim, _ = make_sim(sem, wl, "f32", "hilbert", scatter=sc)
            spc, _, _ = time_steps(torch, sc_sim, min(args.steps, 200), 5)
            lg = leg_summary(sc_sim, spc, f"scatter {sc}")
            out["scatter"][sc] = {"us_per_step": lg["us_per_step"], "gdof_steps_per_s": lg["gdof_steps_per_s"],
                                  "n_colours": sc_sim.info()["n_colours"],
                                  "time_vs_lds_atomic": lg["us_per_step"] / main_leg["us_per_step"]}
            sc_sim.close()
    if "orders" in legs:
        order_keys = ("gdof_steps_per_s", "us_per_step", "hbm_frac", "halo_ratio", "setup_s", "reorder_s",
                      "n_colours")
        out["orders"] = {"hilbert": {k: main_leg[k] for k in order_keys}}
        for order in ("morton", "lex", "random", "connectivity", "distance"):
            log(f"[bench] order {order}")
            so, _ = make_sim(sem, wl, "f32", order)
            spo, _, _ = time_steps(torch, so, min(args.steps, 200), 5)
            lg = leg_summary(so, spo, order)
            out["orders"][order] = {k: lg[k] for k in order_keys}
            so.close()
    if "heun" in legs:
        log("[bench] heun leg: the first-order u-v system with Heun, layered1024 p=4 FP32")
        sh, _ = make_sim(sem, wl, "f32", "hilbert", formulation="heun")
        sph, _, _ = time_steps(torch, sh, min(args.steps, 200), args.warmup)
        out["heun"] = leg_summary(sh, sph, "layered1024 p4 f32 hilbert S=1 first-order Heun")
        out["heun"]["time_ratio_vs_leapfrog"] = sph / (main_leg["us_per_step"] / 1e6)
        sh.close()
    if "tri" in legs:
        # the paper's own element: 250k triangles, p = 5 (21 Blyth-Pozrikidis nodes), the
        # single-layer benchmark shape, in the curve order, the generator order and random
        log("[bench] tri leg: 250k triangles p=5 (the paper's element), FP32 / FP64")
        wt = workloads.workload("tri2000")
        out["tri"] = {}
        for prec, order in (("f32", "hilbert"), ("f32", "lex"), ("f32", "random"), ("f64", "hilbert")):
            st_, _ = make_sim(sem, wt, prec, order)
            spt, _, _ = time_steps(torch, st_, min(args.steps, 200), 10)
            lg = leg_summary(st_, spt, f"tri2000 p5 {prec} {order}")
            lg["n_colours"] = st_.info()["n_colours"]
            out["tri"][f"{prec}_{order}"] = {k: lg[k] for k in (
                "gdof_steps_per_s", "us_per_step", "alg_bytes_per_step", "achieved_GBs", "hbm_frac",
                "halo_ratio", "setup_s", "reorder_s", "n_colours", "n_nodes", "n_elements")}
            st_.close()
    if "graded" in legs:
        log("[bench] graded leg: 1414^2 quads graded 1:8, p=5, FP32, Hilbert / Morton / random")
        wg = workloads.workload("graded1414")
        out["graded"] = {}
        for order in ("hilbert", "morton", "random"):
            sg, _ = make_sim(sem, wg, "f32", order)
            spg, _, _ = time_steps(torch, sg, min(args.steps, 100), 5)
            lg = leg_summary(sg, spg, f"graded1414 p5 f32 {order}")
            out["graded"][order] = {k: lg[k] for k in ("gdof_steps_per_s", "us_per_step", "hbm_frac",
                                                       "halo_ratio", "setup_s", "reorder_s", "n_colours")}
            sg.close()
    if "batch" in legs:
        log("[bench] batch leg: 512^2 p=4, 64 shots FP32 vs single-shot FP64")
        wb = workloads.workload("batch512")
        sb, _ = make_sim(sem, wb, "f32", "hilbert")
        spb, _, _ = time_steps(torch, sb, min(args.steps, 200), 10)
        out["batch64"] = leg_summary(sb, spb, "batch512 p4 f32 hilbert S=64")
        sb.close()
        w1 = workloads.workload("batch512", n_shots=1)
        s1, _ = make_sim(sem, w1, "f64", "hilbert")
        sp1, _, _ = time_steps(torch, s1, min(args.steps, 300), 10)
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
    traffic = headline_traffic() if (args.workload, args.precision, args.order, args.n, args.scatter,
                                      args.formulation) == ("layered1024", "f32", "hilbert", None, "auto",
                                                            "leapfrog") else None
    sec = main_leg["us_per_step"] / 1e6
    # the same step against what it measurably moves and against the device's copy rate
    main_leg["measured_traffic_GBs"] = traffic / sec / 1e9 if traffic else None
    main_leg["measured_traffic_frac_of_peak"] = traffic / sec / 1e9 / HBM_PEAK_GBS if traffic else None
    main_leg["copy_GBs"] = copy_gbs
    main_leg["achieved_frac_of_copy"] = main_leg["achieved_GBs"] / copy_gbs
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
                     "unit": "GB/s", "frac": main_leg["hbm_frac"], "traffic": traffic},
        "cpu_baseline": cpu,
        "main": main_leg,
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
