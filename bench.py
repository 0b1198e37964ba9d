#!/usr/bin/env python3
"""Throughput of the fused FP central-moment stream-collide step on one MI355X.

Workload: 2D Rayleigh-Benard, 1024 x 512 nodes, D2Q9 fluid + D2Q5 thermal,
Ra 1e6, Pr 0.71 (periodic in x, hot bottom, cold top), synthetic seeded
initial temperature; one step = one fused pull-stream-collide launch over the
whole grid (fluid + thermal populations).  The headline line is the FP64
form; the same workload in FP32-deviation storage, and the 3D 256^3
D3Q27 + D3Q7 cavity (FP32 deviations, the HBM-bound case), are reported in
the "extra" object.

Timing: W warm-up steps, then K timed steps bracketed by a device
synchronisation, with HIP events recorded on the stream the kernels are
launched on (torch's current stream).  The roofline object uses the
algorithmic bytes of one launch (every population read once and written
once: 2 (Qf + Qg) sizeof(real) per node) over the average launch duration.

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
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--steps3d", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=36)
    ap.add_argument("--mode", choices=("bench", "single", "copy", "pmc-summary", "precision", "adjoint"),
                    default="bench")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--fetch", help="rocprofv3 --pmc FETCH_SIZE output dir (kernel run)")
    ap.add_argument("--write", help="rocprofv3 --pmc WRITE_SIZE output dir (kernel run)")
    ap.add_argument("--copy-fetch", help="rocprofv3 --pmc FETCH_SIZE output dir (copy run)")
    ap.add_argument("--copy-write", help="rocprofv3 --pmc WRITE_SIZE output dir (copy run)")
    ap.add_argument("--kernel-regex", default="step_kernel")
    ap.add_argument("--key", default="rb2d_1024x512_f64")
    ap.add_argument("--workload", default="rb2d_1024x512")
    ap.add_argument("--precision", default="f64")
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


def kernel_fingerprint(kind="step"):
    """sha256 over the sources of the step kernel (kind "step") or of the
    adjoint step kernel (kind "adjoint"), everything they include: counters
    recorded for other sources do not describe the kernel that runs."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_09041_amd", "csrc")
    common = ("fpc_gather.h", "fpc_collide.h", "fpc_kernels.h", "fpc_lattice.h")
    own = ("fpc_step.hip",) if kind == "step" else ("fpc_adjoint.hip", "fpc_adjoint.h")
    for name in own + common:
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


def time_workload(name, precision, steps, warmup, shape=None, pair=None, model="FP", thermal_option="A"):
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation, params_from_workload

    cfg = workloads.config(name)
    if shape is not None:
        cfg["shape"] = tuple(shape)
    if pair is not None:
        cfg["pair"] = pair
    kw = dict(model=model, thermal_option=thermal_option)
    if precision == "f32cond":
        p = params_from_workload(cfg, "f32dev", T_reference="conduction", **kw)
    else:
        p = params_from_workload(cfg, precision, **kw)
    sim = Simulation(p)
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
    per_launch_s = ms * 1e-3 / steps
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
        "achieved_GBs": bytes_per_node * N / per_launch_s / 1e9,
        "nu": d["nu"],
        "unstable": d["unstable"],
    }
    sim.close()
    return out


def adjoint_cost(name, nsteps, every, reps=20):
    """Cost of the adjoint relative to the forward step (FP32-deviation form).

    kernel_ratio: one adjoint_step launch / one forward step launch (HIP events);
    sweep_ratio: the whole checkpointed reverse sweep (segment recompute, state
    saves, adjoint steps) per step / one forward step."""
    import ctypes

    import torch

    import workloads
    from paper_2504_09041_amd import _abi as A
    from paper_2504_09041_amd import adjoint as adj
    from paper_2504_09041_amd.sim import params_from_workload

    cfg = workloads.config(name)
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
        "workload": name, "precision": "f32dev", "steps": nsteps, "checkpoint_every": every,
        "forward_ms_per_step": t_fwd, "adjoint_kernel_ms": t_adj, "sweep_ms_per_step": t_sweep,
        "kernel_ratio": t_adj / t_fwd, "sweep_ratio": t_sweep / t_fwd,
    }


def precision_study(name, nsteps, every, noise=1e-7, shape=None, **overrides):
    """FP32-deviation forms against FP64 on the same run, every `every` steps:
    max |T - T64| / dT and |Nu - Nu64| / |Nu64| for
      f32dev   FP32 deviations from the uniform reference T0,
      f32cond  FP32 deviations from the conduction profile (affine reference),
      f64pert  FP64 from an initial temperature perturbed by `noise` dT
               (uniform noise): the divergence the flow itself produces from
               a perturbation of FP32 rounding size, the yardstick for the
               other two.
    ``shape`` and ``overrides`` (e.g. Pe) change the workload's grid and
    physical parameters."""
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation, params_from_workload

    cfg = workloads.config(name, **({"shape": tuple(shape)} if shape else {}), **overrides)
    dT = cfg["T_hot"] - cfg["T_cold"]
    T = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    Tp = T + noise * dT * torch.tensor(workloads.uniform_field(tuple(T.shape), 77), device="cuda")
    variants = {
        "f64": (params_from_workload(cfg, "f64"), T),
        "f32dev": (params_from_workload(cfg, "f32dev"), T),
        "f32cond": (params_from_workload(cfg, "f32dev", T_reference="conduction"), T),
        "f64pert": (params_from_workload(cfg, "f64"), Tp),
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
        for k in ("f32dev", "f32cond", "f64pert"):
            row[k] = {"max_dT_over_DeltaT": float((out[k][1] - out["f64"][1]).abs().max()) / dT,
                      "rel_dNu": abs(out[k][0] - out["f64"][0]) / abs(out["f64"][0])}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    for s in sims.values():
        s.close()
    return {"workload": name, "shape": list(cfg["shape"]), "noise": noise, "rows": rows,
            **{k: v for k, v in overrides.items()}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, nsteps, nsteps_1t=6):
    """The FP64 CPU oracle on the host cores, on a bounded sample of the same
    workload (nsteps steps of the full grid after its initial collision), with
    all threads and with one thread."""
    import torch

    import workloads
    from oracle import sim as osim
    from oracle.params import params_from_config

    cfg = workloads.config(name)
    prm = params_from_config(cfg)
    N = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    T = torch.tensor(workloads.initial_temperature(cfg))
    f0, g0 = osim.init_state(prm, T)

    def timed(threads, n):
        torch.set_num_threads(threads)
        f, g, _ = osim.step(prm, f0, g0)  # warm-up step (not timed)
        t0 = time.perf_counter()
        osim.run(prm, f, g, n)
        return time.perf_counter() - t0

    threads = os.cpu_count() or 1
    dt = timed(threads, nsteps)
    dt1 = timed(1, nsteps_1t) if nsteps_1t > 0 else None
    torch.set_num_threads(threads)
    return {
        "value": N * nsteps / dt / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{nsteps} FP64 oracle steps of the full {cfg['shape'][0]}x{cfg['shape'][1]} grid "
                  f"({dt:.1f} s, {threads} threads)",
        "value_1_thread": N * nsteps_1t / dt1 / 1e6 if dt1 else None,
        "sample_1_thread": f"{nsteps_1t} steps ({dt1:.1f} s)" if dt1 else None,
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }


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
    if a.mode == "copy":
        print(json.dumps(copy_bandwidth(a.mib, a.reps)))
        return
    if a.mode == "single":
        print(json.dumps(time_workload(a.workload, a.precision, a.steps, a.warmup)))
        return
    if a.mode == "precision":
        print(json.dumps(precision_study(a.workload, a.steps, max(1, a.steps // 50))))
        return
    if a.mode == "adjoint":
        print(json.dumps(adjoint_cost(a.workload, a.steps, max(1, int(round(a.steps ** 0.5))))))
        return
    head = time_workload("rb2d_1024x512", "f64", a.steps, a.warmup)
    extra = {}
    if not a.no_extra:
        extra["rb2d_1024x512_f32dev"] = time_workload("rb2d_1024x512", "f32dev", a.steps, a.warmup)
        extra["rb2d_1024x512_f32cond"] = time_workload("rb2d_1024x512", "f32cond", a.steps, a.warmup)
        extra["dhc3d_256_f32dev"] = time_workload("dhc3d_256", "f32dev", a.steps3d, max(5, a.warmup // 10))
        extra["rb3d_128_f32dev"] = time_workload("rb3d_128", "f32dev", 5 * a.steps3d, max(5, a.warmup // 10))
        # the same 2D physics on a grid whose state (3.8 GB) does not fit the
        # last-level cache: a pure-HBM figure for the FP64 kernel
        extra["rb2d_4096x4096_f64"] = time_workload("rb2d_1024x512", "f64", a.steps3d, max(5, a.warmup // 10),
                                                    shape=(4096, 4096, 1))
        # the 3D cavity at 64^3 in FP64 and the 512^2 mixed-convection case in
        # FP32 (forward step of the adjoint workload)
        extra["dhc3d_64_f64"] = time_workload("dhc3d_256", "f64", 5 * a.steps3d, max(5, a.warmup // 10),
                                              shape=(64, 64, 64))
        extra["mixed2d_512_f32dev"] = time_workload("mixed2d_512", "f32dev", a.steps, a.warmup)
        # the 64 x 64 cavity: launch-bound (4096 nodes per launch)
        extra["dhc2d_64_f64"] = time_workload("dhc2d_64", "f64", a.steps, a.warmup)
        extra["copy_4GiB"] = copy_bandwidth(4096, 20)
        # the paper's own thermal lattices (FP64), and the MCM comparator on the
        # headline workload: same step structure, more (or the same) bytes
        extra["rb2d_1024x512_f64_D2Q9thermal"] = time_workload("rb2d_1024x512", "f64", a.steps, a.warmup,
                                                               pair="D2Q9-D2Q9")
        extra["rb3d_128_f64_D3Q15thermal"] = time_workload("rb3d_128", "f64", a.steps3d, max(5, a.warmup // 10),
                                                           pair="D3Q27-D3Q15")
        extra["rb2d_1024x512_f64_MCM"] = time_workload("rb2d_1024x512", "f64", a.steps, a.warmup, model="MCM")
        # FP32 against FP64 over the workload's full run (the precision half of
        # the metric): errors of T and of the bottom-wall Nu at the end
        cfg_steps = 50000
        st = precision_study("rb2d_1024x512", cfg_steps, cfg_steps // 5)
        last = st["rows"][-1]
        extra["fp32_vs_fp64_rb2d_1024x512"] = {
            "steps": cfg_steps, "nu_f64": last["nu_f64"],
            "f32dev_uniform_ref": last["f32dev"], "f32dev_conduction_ref": last["f32cond"],
            "f64_perturbed_1e-7": last["f64pert"],
            "bars": {"max_dT_over_DeltaT": 1e-4, "rel_dNu": 1e-3},
        }
        # the 3D cavity's FP32 run against FP64 at 64^3 over its 20k steps
        st = precision_study("dhc3d_256", 20000, 20000, shape=(64, 64, 64))
        last = st["rows"][-1]
        extra["fp32_vs_fp64_dhc3d_64"] = {
            "steps": 20000, "nu_f64": last["nu_f64"], "f32dev_uniform_ref": last["f32dev"],
            "f32dev_conduction_ref": last["f32cond"], "f64_perturbed_1e-7": last["f64pert"],
        }
        # the lid-driven mixed-convection cavity over its Pe range (10k steps)
        for pe in (1e3, 1e4, 1e5):
            st = precision_study("mixed2d_512", 10000, 10000, Pe=pe)
            last = st["rows"][-1]
            extra[f"fp32_vs_fp64_mixed2d_512_Pe{pe:.0e}"] = {
                "steps": 10000, "Pe": pe, "nu_f64": last["nu_f64"], "f32dev_uniform_ref": last["f32dev"],
                "f32dev_conduction_ref": last["f32cond"], "f64_perturbed_1e-7": last["f64pert"],
            }
    if not a.no_extra and not a.no_adjoint:
        extra["adjoint_mixed2d_512_f32dev"] = adjoint_cost("mixed2d_512", 400, 100)
        extra["adjoint_rb3d_128_f32dev"] = adjoint_cost("rb3d_128", 64, 8)
    tr = _traffic_record().get("rb2d_1024x512_f64")
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
        # fraction of what a plain elementwise copy attains on this device
        "frac_of_copy": head["achieved_GBs"] / copy["GBs"] if copy else None,
    }
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline("rb2d_1024x512", a.cpu_sample_steps)
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "rb2d_1024x512: 2D Rayleigh-Benard 1024x512, D2Q9+D2Q5 FP central-moment LBM, "
                        "Ra=1e6, Pr=0.71, FP64",
            "lattice": "D2Q9+D2Q5",
            "grid": [1024, 512],
            "precision": "f64",
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
