#!/usr/bin/env python3
"""Throughput of the fused FP central-moment stream-collide step on one MI355X.

Headline workload: the 3D differentially heated cube, 256^3 nodes, D3Q27
fluid + D3Q7 thermal, Ra 1e6, Pr 0.71 (hot and cold x walls, adiabatic
no-slip elsewhere), FP32-deviation storage with the library's default
storage reference, synthetic seeded initial temperature.  Its 4.56 GB of
state streams through HBM on every step.  One step = one fused
pull-stream-collide launch over the whole grid (fluid + thermal
populations).  The other workloads (the 2D Rayleigh-Benard case whose state
stays in the last-level cache, the FP64 forms, the paper's own thermal
lattices, the precision and adjoint studies) are in the "extra" object.

Timing: W warm-up steps, then K timed steps bracketed by a device
synchronisation, with HIP events recorded on the stream the kernels are
launched on (torch's current stream).  The roofline object uses the
algorithmic bytes of one launch (every population read once and written
once: 2 (Qf + Qg) sizeof(real) = 272 B per node) over the average launch
duration.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Profiling helpers (used for the rocprofv3 summaries under profiles/):
    python bench.py --mode single --workload dhc3d_256 --precision f32dev --steps 5
        runs one workload only (init + W warm-up + K steps) and prints its timing;
    python bench.py --mode copy --mib 4096 --reps 10
        a plain device copy (torch) of a buffer of that size: the attainable
        read+write bandwidth and the reference for the HBM byte counters.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--steps2d", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--shape", type=int, nargs=3, help="grid (nx ny nz) of --mode single instead of the workload's")
    ap.add_argument("--pair", help="lattice pair of --mode single / precision instead of the workload's "
                                   "(D2Q9-D2Q5, D2Q9-D2Q9, D3Q27-D3Q7, D3Q27-D3Q15)")
    ap.add_argument("--no-multistep", action="store_true",
                    help="forbid fpc_step's single-launch multi-step path (small grids)")
    ap.add_argument("--cpu-sample-steps", type=int, default=24)
    ap.add_argument("--mode", choices=("bench", "single", "copy", "pmc-summary", "trace-summary", "precision", "adjoint",
                                       "objective", "diagnostics"),
                    default="bench")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--fetch", help="rocprofv3 --pmc FETCH_SIZE output dir (kernel run)")
    ap.add_argument("--write", help="rocprofv3 --pmc WRITE_SIZE output dir (kernel run)")
    ap.add_argument("--copy-fetch", help="rocprofv3 --pmc FETCH_SIZE output dir (copy run)")
    ap.add_argument("--copy-write", help="rocprofv3 --pmc WRITE_SIZE output dir (copy run)")
    ap.add_argument("--kernel-regex", default="step_kernel")
    ap.add_argument("--trace", help="rocprofv3 --kernel-trace csv output dir (trace-summary)")
    ap.add_argument("--top", type=int, default=45, help="rows of the trace summary")
    ap.add_argument("--key", default="dhc3d_256_f32dev")
    ap.add_argument("--workload", default="dhc3d_256")
    ap.add_argument("--precision", default="f32dev")
    ap.add_argument("--mib", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=10)
    return ap.parse_args()


def copy_bandwidth(mib, reps):
    import torch

    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    # an elementwise kernel (torch's vectorised streaming loop), not the
    # runtime's blit copy
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * n * 4
    return {"mode": "copy", "bytes_read_plus_written": nbytes, "ms_per_copy": ms,
            "GBs": nbytes / (ms * 1e-3) / 1e9}


def fingerprint_sources(kind="step"):
    """Source files of the step kernel (kind "step") or of the adjoint step
    kernels whose counters are recorded (kind "adjoint": the D2Q9 + D2Q5 and
    D3Q27 + D3Q7 pairs), with everything they include."""
    common = ("fpc_gather.h", "fpc_collide.h", "fpc_kernels.h", "fpc_lattice.h")
    own = ("fpc_step.hip",) if kind == "step" else ("fpc_adjoint.hip", "fpc_adjoint_d3q7.hip", "fpc_adjoint_kernels.h",
                                                     "fpc_adjoint.h")
    return own + common


def kernel_fingerprint(kind="step"):
    """sha256 over fingerprint_sources(kind): counters recorded for other
    sources do not describe the kernel that runs."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_09041_amd", "csrc")
    for name in fingerprint_sources(kind):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _traffic_record():
    """HBM bytes per launch measured with rocprofv3 counters, if recorded."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def _pmc_per_dispatch(d, regex):
    """Mean counter value (KiB, summed over the counter's instances) per
    dispatch of the kernels matching ``regex`` in a rocprofv3 csv directory."""
    import csv
    import glob
    import re

    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    per = {}
    for r in csv.DictReader(open(path)):
        if re.search(regex, r["Kernel_Name"]):
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    vals = sorted(per.values())
    # drop the first dispatch of a run when it differs (initial collision)
    return sum(vals[len(vals) // 2:]) / len(vals[len(vals) // 2:]), len(vals)


def trace_summary(a):
    """Markdown table of a rocprofv3 kernel trace: dispatches grouped by kernel
    and launch grid, with calls, average / median duration and total time."""
    import csv
    import glob
    import statistics

    path = glob.glob(os.path.join(a.trace, "**", "*kernel_trace.csv"), recursive=True)[0]
    groups = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        grid = "x".join(r["Grid_Size_" + k] for k in "XYZ")
        block = "x".join(r["Workgroup_Size_" + k] for k in "XY")
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3  # us
        groups.setdefault((name, grid, block), []).append(dur)
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[: a.top]
    out = ["| kernel | grid | block | calls | avg us | median us | total ms |", "|---|---|---|---|---|---|---|"]
    for (name, grid, block), d in rows:
        short = name if len(name) <= 150 else name[:150] + "..."
        out.append(f"| `{short}` | {grid} | {block} | {len(d)} | {sum(d) / len(d):.2f} | "
                   f"{statistics.median(d):.2f} | {sum(d) * 1e-3:.1f} |")
    return "\n".join(out)


def pmc_summary(a):
    """Scale the TCC byte counters by what they read for a plain copy of
    known size and record bytes per launch in profiles/traffic.json."""
    copy_bytes = a.mib * 1024 * 1024
    cf, _ = _pmc_per_dispatch(a.copy_fetch, "elementwise")
    cw, _ = _pmc_per_dispatch(a.copy_write, "elementwise")
    kf, nf = _pmc_per_dispatch(a.fetch, a.kernel_regex)
    kw, nw = _pmc_per_dispatch(a.write, a.kernel_regex)
    sf = copy_bytes / (cf * 1024.0)
    sw = copy_bytes / (cw * 1024.0)
    rec = {
        "fetch_bytes": kf * 1024.0 * sf, "write_bytes": kw * 1024.0 * sw,
        "fetch_scale": sf, "write_scale": sw, "dispatches": [nf, nw],
    }
    rec["traffic_bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
    rec["sources"] = kernel_fingerprint("adjoint" if "adjoint" in a.kernel_regex else "step")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    allrec = _traffic_record()
    allrec[a.key] = rec
    with open(path, "w") as fh:
        json.dump(allrec, fh, indent=1, sort_keys=True)
    return rec


def workload_params(cfg, precision, **kw):
    """C parameters of a workload in one of the forms: "f64"; "f32dev" (FP32
    deviations, the library's default storage reference: the conduction
    profile between a pair of Dirichlet walls); "f32uni" (FP32 deviations
    from the uniform T0, the literal g - w^T T0 form); "f32cond" (the
    conduction reference along the workload's L axis, set explicitly)."""
    from paper_2504_09041_amd.sim import params_from_workload

    if precision == "f32uni":
        return params_from_workload(cfg, "f32dev", T_reference="uniform", **kw)
    if precision == "f32cond":
        return params_from_workload(cfg, "f32dev", T_reference="conduction", **kw)
    return params_from_workload(cfg, precision, **kw)


def time_workload(name, precision, steps, warmup, shape=None, pair=None, model="FP", thermal_option="A",
                  multistep=True):
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation

    cfg = workloads.config(name)
    if shape is not None:
        cfg["shape"] = tuple(shape)
    if pair is not None:
        cfg["pair"] = pair
    p = workload_params(cfg, precision, model=model, thermal_option=thermal_option)
    sim = Simulation(p)
    sim.set_multistep(multistep)
    T = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    sim.init(T)
    del T
    sim.step(warmup)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d = sim.diagnostics(cfg["nu_face"])
    N = sim.N
    elem = 8 if precision == "f64" else 4
    bytes_per_node = 2 * (sim.Qf + sim.Qg) * elem
    per_step_s = ms * 1e-3 / steps
    launches = sim.multistep_launches
    out = {
        "workload": name,
        "pair": cfg["pair"],
        "model": model,
        "precision": precision,
        "shape": list(cfg["shape"]),
        "nodes": N,
        "steps": steps,
        "ms_per_step": ms / steps,
        "wall_s": wall,
        "mlups": N * steps / (ms * 1e-3) / 1e6,
        "bytes_per_node": bytes_per_node,
        "achieved_GBs": bytes_per_node * N / per_step_s / 1e9,
        "multistep_launches": launches,
        "nu": d["nu"],
        "unstable": d["unstable"],
    }
    sim.close()
    return out


def adjoint_cost(name, nsteps, every, reps=20, pair=None):
    """Cost of the adjoint relative to the forward step (FP32-deviation form;
    ``pair`` another lattice pair than the workload's).

    kernel_ratio: one adjoint_step launch / one forward step launch (HIP events);
    sweep_ratio: the whole checkpointed reverse sweep (segment recompute, state
    saves, adjoint steps) per step / one forward step."""
    import ctypes

    import torch

    import workloads
    from paper_2504_09041_amd import _abi as A
    from paper_2504_09041_amd import adjoint as adj
    from paper_2504_09041_amd.sim import params_from_workload

    cfg = workloads.config(name, **({"pair": pair} if pair else {}))
    p = params_from_workload(cfg, "f32dev")
    if name.startswith("mixed"):
        obj = adj.WallNusselt(cfg["nu_face"], nsteps // 2, nsteps)
        solver = adj.AdjointSolver(p, nsteps, every, obj, theta_face=cfg.get("grad_face", 2))
    else:
        obj = adj.KineticEnergy(nsteps)
        solver = adj.AdjointSolver(p, nsteps, every, obj)
    T = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    solver.forward(None, T)
    sim = solver.sim
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    # forward step alone
    sim.step(5)
    e0, e1 = ev(), ev()
    torch.cuda.synchronize()
    e0.record()
    sim.step(reps)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / reps
    # adjoint step alone
    S = sim.save()
    lam = sim.new_adjoint()
    lam2 = sim.new_adjoint()
    lib = A.load()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    for _ in range(3):
        lib.fpc_adjoint_step(sim.handle, vp(S), vp(lam), vp(lam2), None, ctypes.c_double(1.0), None)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        A.check(lib.fpc_adjoint_step(sim.handle, vp(S), vp(lam), vp(lam2), None, ctypes.c_double(1.0), None),
                "fpc_adjoint_step")
        lam, lam2 = lam2, lam
    e1.record()
    torch.cuda.synchronize()
    t_adj = e0.elapsed_time(e1) / reps
    # whole reverse sweep
    solver.forward(None, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.backward()
    torch.cuda.synchronize()
    t_sweep = (time.perf_counter() - t0) * 1e3 / nsteps
    sim.close()
    return {
        "workload": name, "pair": cfg["pair"], "precision": "f32dev", "steps": nsteps, "checkpoint_every": every,
        "forward_ms_per_step": t_fwd, "adjoint_kernel_ms": t_adj, "sweep_ms_per_step": t_sweep,
        "kernel_ratio": t_adj / t_fwd, "sweep_ratio": t_sweep / t_fwd,
    }


BARS = {"max_dT_over_DeltaT": 1e-4, "rel_dNu": 1e-3}


def precision_study(name, nsteps, every, noise=1e-7, shape=None, **overrides):
    """FP32-deviation forms against FP64 on the same run, every `every` steps:
    max |T - T64| / dT and |Nu - Nu64| / |Nu64| for
      f32dev   FP32 deviations with the library's default storage reference
               (the conduction profile between the Dirichlet walls),
      f32uni   FP32 deviations from the uniform reference T0 (the literal
               g - w^T T0 form),
      f64pert  FP64 from an initial temperature perturbed by `noise` dT
               (uniform noise): the divergence the flow itself produces from
               a perturbation of FP32 rounding size, the yardstick for the
               other two.
    ``shape`` and ``overrides`` (e.g. Pe) change the workload's grid and
    physical parameters."""
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation

    cfg = workloads.config(name, **({"shape": tuple(shape)} if shape else {}), **overrides)
    dT = cfg["T_hot"] - cfg["T_cold"]
    T = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    Tp = T + noise * dT * torch.tensor(workloads.uniform_field(tuple(T.shape), 77), device="cuda")
    variants = {
        "f64": (workload_params(cfg, "f64"), T),
        "f32dev": (workload_params(cfg, "f32dev"), T),
        "f32uni": (workload_params(cfg, "f32uni"), T),
        "f64pert": (workload_params(cfg, "f64"), Tp),
    }
    sims = {}
    for k, (p, T_init) in variants.items():
        s = Simulation(p)
        s.init(T_init)
        sims[k] = s
    rows = []
    for n in range(every, nsteps + 1, every):
        out = {}
        for k, s in sims.items():
            s.step(every)
            out[k] = (s.diagnostics(cfg["nu_face"])["nu"], s.macros()["T"])
        row = {"step": n, "nu_f64": out["f64"][0]}
        for k in ("f32dev", "f32uni", "f64pert"):
            row[k] = {"max_dT_over_DeltaT": float((out[k][1] - out["f64"][1]).abs().max()) / dT,
                      "rel_dNu": abs(out[k][0] - out["f64"][0]) / abs(out["f64"][0])}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    for s in sims.values():
        s.close()
    return {"workload": name, "shape": list(cfg["shape"]), "noise": noise, "rows": rows,
            **{k: v for k, v in overrides.items()}}


def precision_summary(st, steps, **extra):
    """Worst errors of each form over the study's rows, with pass flags
    against the bars (1e-4 dT on T, 1e-3 relative on Nu)."""
    out = {"steps": steps, **extra, "nu_f64": st["rows"][-1]["nu_f64"], "bars": BARS}
    for k, label in (("f32dev", "f32dev_default_ref"), ("f32uni", "f32dev_uniform_ref"),
                     ("f64pert", "f64_perturbed_1e-7")):
        worst = {m: max(r[k][m] for r in st["rows"]) for m in BARS}
        rec = {"worst_over_run": worst, "last": st["rows"][-1][k]}
        if k != "f64pert":
            rec["pass"] = all(worst[m] <= BARS[m] for m in BARS)
        out[label] = rec
    return out


def objective_cost(name, nsteps, reps=3):
    """Cost of accumulating the wall-Nusselt objective during the forward run
    (fpc_step_nusselt, fused into the step kernel) against plain steps: the
    forward over the workload's J window, FP32 deviations."""
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation

    cfg = workloads.config(name)
    sim = Simulation(workload_params(cfg, "f32dev"))
    sim.init(torch.tensor(workloads.initial_temperature(cfg), device="cuda"))
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    sim.step(100)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    best = {}
    for kind in ("plain", "nusselt") * reps:
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record()
        if kind == "plain":
            sim.step(nsteps)
        else:
            sim.step_nusselt(nsteps, cfg["nu_face"], 1.0 / nsteps, acc)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / nsteps
        best[kind] = min(best.get(kind, float("inf")), ms)
    sim.close()
    return {"workload": name, "precision": "f32dev", "steps": nsteps, "plain_ms_per_step": best["plain"],
            "objective_ms_per_step": best["nusselt"], "ratio": best["nusselt"] / best["plain"],
            "target_ratio": 1.3}


def diagnostics_cost(name, precision, reps=20, rounds=3):
    """Cost of the diagnostics of a step: a plain step, a step whose kernel
    also reduces the diagnostics of the state it writes (fpc_step_diagnostics,
    1 step per call), and a plain step followed by the separate diagnostics
    pass over the stored state (fpc_diagnostics_noalloc, which reads the state
    once more); HIP events on the stream, best of `rounds`."""
    import ctypes

    import torch

    import workloads
    from paper_2504_09041_amd import _abi as A
    from paper_2504_09041_amd.sim import Simulation

    cfg = workloads.config(name)
    sim = Simulation(workload_params(cfg, precision))
    sim.init(torch.tensor(workloads.initial_temperature(cfg), device="cuda"))
    sim.step(10)
    lib = A.load()
    face = cfg["nu_face"]
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    pout = ctypes.c_void_p(out.data_ptr())
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    best = {}
    for kind in ("plain", "fused", "separate") * rounds:
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            if kind == "plain":
                sim.step(1)
            elif kind == "fused":
                sim.step_diagnostics(1, face, out)
            else:
                sim.step(1)
                A.check(lib.fpc_diagnostics_noalloc(sim.handle, face, pout), "fpc_diagnostics_noalloc")
        e1.record()
        torch.cuda.synchronize()
        best[kind] = min(best.get(kind, float("inf")), e0.elapsed_time(e1) / reps)
    d = out.cpu().tolist()
    sim.close()
    return {"workload": name, "precision": precision, "shape": list(cfg["shape"]),
            "plain_step_ms": best["plain"], "fused_step_diagnostics_ms": best["fused"],
            "step_then_diagnostics_pass_ms": best["separate"],
            "fused_over_plain": best["fused"] / best["plain"],
            "separate_over_plain": best["separate"] / best["plain"],
            "last": {"nu": d[0], "ke": d[1], "sumT": d[2], "umax": d[3], "non_finite": d[4]}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nsteps3d, nsteps_1t=3, config1=True, gradients=True):
    """The FP64 CPU oracle on the host cores, on bounded samples:
    value: nsteps3d steps of the 3D cube at 32^3 (D3Q27 + D3Q7, the headline
    lattice pair) after its initial collision, all threads; a few steps on
    one thread; the 64 x 64 cavity over its full 2000 steps; and the
    oracle's reference gradients (torch autograd through the FP64 oracle) at
    16^3 (3D Rayleigh-Benard, KE objective) and 32 x 32 (lid-driven mixed
    convection, windowed Nusselt objective)."""
    import torch

    import workloads
    from oracle import gradient as ograd
    from oracle import sim as osim
    from oracle.params import params_from_config

    threads = os.cpu_count() or 1

    def timed_run(name, shape, n, nthreads):
        cfg = workloads.config(name, shape=shape)
        prm = params_from_config(cfg)
        T = torch.tensor(workloads.initial_temperature(cfg))
        f, g = osim.init_state(prm, T)
        torch.set_num_threads(nthreads)
        f, g, _ = osim.step(prm, f, g)  # warm-up step (not timed)
        t0 = time.perf_counter()
        osim.run(prm, f, g, n)
        dt = time.perf_counter() - t0
        torch.set_num_threads(threads)
        N = shape[0] * shape[1] * shape[2]
        return N * n / dt / 1e6, dt

    mlups, dt = timed_run("dhc3d_256", (32, 32, 32), nsteps3d, threads)
    out = {
        "value": mlups,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{nsteps3d} FP64 oracle steps of the 3D cube at 32^3 (D3Q27+D3Q7, the headline lattice pair; "
                  f"{dt:.1f} s, {threads} threads)",
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }
    if nsteps_1t > 0:
        m1, d1 = timed_run("dhc3d_256", (32, 32, 32), nsteps_1t, 1)
        out["value_1_thread"] = m1
        out["sample_1_thread"] = f"{nsteps_1t} steps of the same 32^3 cube on 1 thread ({d1:.1f} s)"
    if config1:
        m, d = timed_run("dhc2d_64", (64, 64, 1), 2000, threads)
        out["cavity_64x64_full_run"] = {"mlups": m, "seconds": d, "steps": 2000, "threads": threads}
    if gradients:
        cfg = workloads.config("rb3d_128", shape=(16, 16, 16))
        prm = params_from_config(cfg)
        T = torch.tensor(workloads.initial_temperature(cfg))
        t0 = time.perf_counter()
        ograd.gradient(prm, T, 20, "ke", at=20)
        d3 = time.perf_counter() - t0
        cfg = workloads.config("mixed2d_512", shape=(32, 32, 1))
        prm = params_from_config(cfg)
        T = torch.tensor(workloads.initial_temperature(cfg))
        th = torch.full((1, 32), cfg["faces"][2]["T"], dtype=torch.float64)
        t0 = time.perf_counter()
        ograd.gradient(prm, T, 40, "nu", face=cfg["nu_face"], window=(20, 40), theta_face=2, theta=th)
        d2 = time.perf_counter() - t0
        out["reference_gradient"] = {
            "rb3d_16^3_ke_20_steps": {"seconds": d3, "seconds_per_step": d3 / 20},
            "mixed2d_32x32_nu_40_steps": {"seconds": d2, "seconds_per_step": d2 / 40},
            "threads": threads,
        }
    return out


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {a.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if a.mode == "pmc-summary":
        print(json.dumps(pmc_summary(a)))
        return
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.mode == "trace-summary":
        print(trace_summary(a))
        return
    if a.mode == "copy":
        print(json.dumps(copy_bandwidth(a.mib, a.reps)))
        return
    if a.mode == "single":
        print(json.dumps(time_workload(a.workload, a.precision, a.steps, a.warmup, shape=a.shape, pair=a.pair,
                                       multistep=not a.no_multistep)))
        return
    if a.mode == "precision":
        kw = {"pair": a.pair} if a.pair else {}
        print(json.dumps(precision_study(a.workload, a.steps, max(1, a.steps // 50), shape=a.shape, **kw)))
        return
    if a.mode == "adjoint":
        print(json.dumps(adjoint_cost(a.workload, a.steps, max(1, int(round(a.steps ** 0.5))), pair=a.pair)))
        return
    if a.mode == "objective":
        print(json.dumps(objective_cost(a.workload, a.steps)))
        return
    if a.mode == "diagnostics":
        print(json.dumps(diagnostics_cost(a.workload, a.precision)))
        return
    head = time_workload("dhc3d_256", "f32dev", a.steps, a.warmup)
    extra = {}
    if not a.no_extra:
        n2, w2 = a.steps2d, max(20, a.steps2d // 20)
        n3, w3 = max(20, a.steps // 2), 10
        # the 2D Rayleigh-Benard workload: its state (117 MB in FP64, 59 MB in
        # FP32) stays in the 256 MB last-level cache, so it runs faster than
        # a copy through HBM
        extra["rb2d_1024x512_f64_llc_resident"] = time_workload("rb2d_1024x512", "f64", n2, w2)
        extra["rb2d_1024x512_f32dev_llc_resident"] = time_workload("rb2d_1024x512", "f32dev", n2, w2)
        extra["rb2d_1024x512_f32uni_llc_resident"] = time_workload("rb2d_1024x512", "f32uni", n2, w2)
        extra["dhc3d_256_f32uni"] = time_workload("dhc3d_256", "f32uni", n3, w3)
        extra["rb3d_128_f32dev"] = time_workload("rb3d_128", "f32dev", 5 * n3, w3)
        # the same 2D physics on a grid whose state (3.8 GB) does not fit the
        # last-level cache: a pure-HBM figure for the FP64 kernel
        extra["rb2d_4096x4096_f64"] = time_workload("rb2d_1024x512", "f64", n3, w3, shape=(4096, 4096, 1))
        # the 3D cavity at 64^3 in FP64 and the 512^2 mixed-convection case in
        # FP32 (forward step of the adjoint workload)
        extra["dhc3d_64_f64"] = time_workload("dhc3d_256", "f64", 5 * n3, w3, shape=(64, 64, 64))
        extra["mixed2d_512_f32dev"] = time_workload("mixed2d_512", "f32dev", n2, w2)
        # the 64 x 64 cavity: latency-bound (4096 nodes); fpc_step runs it with
        # up to 1024 steps per cooperative launch, and here also with one
        # launch per step
        extra["dhc2d_64_f64"] = time_workload("dhc2d_64", "f64", n2, w2)
        extra["dhc2d_64_f64_per_step_launches"] = time_workload("dhc2d_64", "f64", n2, w2, multistep=False)
        extra["copy_4GiB"] = copy_bandwidth(4096, 20)
        # the paper's own thermal lattices (FP64), and the MCM comparator on the
        # 2D workload: same step structure, more (or the same) bytes
        extra["rb2d_1024x512_f64_D2Q9thermal"] = time_workload("rb2d_1024x512", "f64", n2, w2, pair="D2Q9-D2Q9")
        extra["rb3d_128_f64_D3Q15thermal"] = time_workload("rb3d_128", "f64", n3, w3, pair="D3Q27-D3Q15")
        extra["rb2d_1024x512_f32dev_D2Q9thermal"] = time_workload("rb2d_1024x512", "f32dev", n2, w2,
                                                                  pair="D2Q9-D2Q9")
        extra["rb3d_128_f32dev_D3Q15thermal"] = time_workload("rb3d_128", "f32dev", n3, w3, pair="D3Q27-D3Q15")
        extra["rb2d_1024x512_f64_MCM"] = time_workload("rb2d_1024x512", "f64", n2, w2, model="MCM")
        # context, not a target: the paper's only performance figure is its
        # C++/MPI code on 512 CPU cores for a 128^3 D3Q27 + D3Q15 run, 5e6
        # steps in about 30.7 h (Sec. 6.2), i.e. about 94.9 MLUPS
        r15 = extra["rb3d_128_f64_D3Q15thermal"]
        extra["paper_cpu_cluster_context_128cube_D3Q15"] = {
            "paper_mlups_512_cores": 2097152 * 5e6 / (30.7 * 3600) / 1e6,
            "this_gpu_mlups_f64": r15["mlups"],
            "this_gpu_mlups_f32dev": extra["rb3d_128_f32dev_D3Q15thermal"]["mlups"],
            "ratio_f64": r15["mlups"] / (2097152 * 5e6 / (30.7 * 3600) / 1e6),
            "note": "other hardware and precision not stated in the paper; context only",
        }
        # the wall-Nusselt objective accumulated during the forward run of the
        # lid-driven cavity's J window (steps 5000-10000)
        extra["objective_forward_mixed2d_512"] = objective_cost("mixed2d_512", 5001)
        # a step that also returns the diagnostics of the state it writes,
        # against a plain step and a step plus the separate diagnostics pass
        extra["diagnostics_dhc3d_256_f32dev"] = diagnostics_cost("dhc3d_256", "f32dev")
        # FP32 against FP64 over the workloads' full runs (the precision half
        # of the metric): worst errors of T and of the wall Nu, pass flags
        st = precision_study("rb2d_1024x512", 50000, 5000)
        extra["fp32_vs_fp64_rb2d_1024x512"] = precision_summary(st, 50000)
        st = precision_study("dhc3d_256", 20000, 5000, shape=(64, 64, 64))
        extra["fp32_vs_fp64_dhc3d_64"] = precision_summary(st, 20000)
        # the FP32 deviation form on the paper's own thermal lattices
        st = precision_study("rb2d_1024x512", 50000, 5000, pair="D2Q9-D2Q9")
        extra["fp32_vs_fp64_rb2d_1024x512_D2Q9thermal"] = precision_summary(st, 50000)
        st = precision_study("dhc3d_256", 20000, 5000, shape=(64, 64, 64), pair="D3Q27-D3Q15")
        extra["fp32_vs_fp64_dhc3d_64_D3Q15thermal"] = precision_summary(st, 20000)
        for pe in (1e3, 1e4, 1e5):
            st = precision_study("mixed2d_512", 10000, 5000, Pe=pe)
            extra[f"fp32_vs_fp64_mixed2d_512_Pe{pe:.0e}"] = precision_summary(st, 10000, Pe=pe)
    if not a.no_extra and not a.no_adjoint:
        extra["adjoint_mixed2d_512_f32dev"] = adjoint_cost("mixed2d_512", 400, 100)
        extra["adjoint_rb3d_128_f32dev"] = adjoint_cost("rb3d_128", 64, 8)
        # the same on the paper's thermal lattices (general-rate adjoint build)
        extra["adjoint_mixed2d_512_f32dev_D2Q9thermal"] = adjoint_cost("mixed2d_512", 400, 100, pair="D2Q9-D2Q9")
        extra["adjoint_rb3d_128_f32dev_D3Q15thermal"] = adjoint_cost("rb3d_128", 64, 8, pair="D3Q27-D3Q15")
    tr = _traffic_record().get("dhc3d_256_f32dev")
    if tr and tr.get("sources") != kernel_fingerprint():
        tr = None  # the kernels changed since the counters were taken
    copy = extra.get("copy_4GiB")
    roof = {
        "bound": "hbm",
        "achieved": head["achieved_GBs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": head["achieved_GBs"] / HBM_PEAK_GBS,
        # HBM-side bytes per launch from the scaled FETCH_SIZE + WRITE_SIZE counters
        "traffic": tr["traffic_bytes"] if tr else None,
        "algorithmic_bytes": head["bytes_per_node"] * head["nodes"],
        "bytes_per_node": head["bytes_per_node"],
        # fraction of what a plain elementwise copy of 4 GiB attains on this device
        "frac_of_copy": head["achieved_GBs"] / copy["GBs"] if copy else None,
    }
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(a.cpu_sample_steps)
    line = {
        "metric": "MLUPS (fluid+thermal) & % HBM roofline; FP32 vs FP64 at stated Nu error; adjoint/fwd",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "dhc3d_256: 3D differentially heated cube 256^3, D3Q27+D3Q7 FP central-moment LBM, "
                        "Ra=1e6, Pr=0.71, FP32-deviation storage (default conduction reference)",
            "lattice": "D3Q27+D3Q7",
            "grid": [256, 256, 256],
            "precision": "f32dev",
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
