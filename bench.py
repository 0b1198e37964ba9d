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
    ap.add_argument("--cpu-sample-steps", type=int, default=12)
    return ap.parse_args()


def _traffic_record():
    """HBM bytes per launch measured with rocprofv3 counters, if recorded."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def time_workload(name, precision, steps, warmup, shape=None):
    import torch

    import workloads
    from paper_2504_09041_amd.sim import Simulation, params_from_workload

    cfg = workloads.config(name)
    if shape is not None:
        cfg["shape"] = tuple(shape)
    p = params_from_workload(cfg, precision)
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


def cpu_baseline(name, nsteps):
    """The FP64 CPU oracle on the host cores, on a bounded sample of the same
    workload (nsteps steps of the full grid after its initial collision)."""
    import torch

    import workloads
    from oracle import sim as osim
    from oracle.params import params_from_config

    torch.set_num_threads(os.cpu_count() or 1)
    cfg = workloads.config(name)
    prm = params_from_config(cfg)
    T = torch.tensor(workloads.initial_temperature(cfg))
    f, g = osim.init_state(prm, T)
    f, g, _ = osim.step(prm, f, g)  # warm-up step (not timed)
    t0 = time.perf_counter()
    f, g, _ = osim.run(prm, f, g, nsteps)
    dt = time.perf_counter() - t0
    N = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    return {
        "value": N * nsteps / dt / 1e6,
        "unit": "MLUPS",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": f"{nsteps} FP64 oracle steps of the full {cfg['shape'][0]}x{cfg['shape'][1]} grid "
                  f"({dt:.1f} s)",
    }


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); "
              "multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    head = time_workload("rb2d_1024x512", "f64", a.steps, a.warmup)
    extra = {}
    if not a.no_extra:
        extra["rb2d_1024x512_f32dev"] = time_workload("rb2d_1024x512", "f32dev", a.steps, a.warmup)
        extra["dhc3d_256_f32dev"] = time_workload("dhc3d_256", "f32dev", a.steps3d, max(5, a.warmup // 10))
    traffic = _traffic_record().get("step2d_f64_rb2d_1024x512")
    roof = {
        "bound": "hbm",
        "achieved": head["achieved_GBs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": head["achieved_GBs"] / HBM_PEAK_GBS,
        "traffic": traffic,
    }
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline("rb2d_1024x512", a.cpu_sample_steps)
    line = {
        "metric": "MLUPS (fluid+thermal)",
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
