"""Numerical stability of the FP central-moment model against the Maxwellian
central-moment comparator (MCM), the study of Sec. 7.

The set-up is the lid-driven cube with a hot moving top, a cold bottom and
adiabatic sides (workload ``mixed3d_64``).  The D3Q27 fluid is coupled to the
paper's D3Q15 thermal lattice, in FP64.  For a grid L^3, a Mach number
Ma = sqrt(3) U0 and a Prandtl number Pr, the thermal diffusivity alpha is
lowered (Pe = U0 L / alpha raised, with nu = Pr alpha) until the run no
longer survives ``steps`` time steps.  A run fails when the watchdog of
fpc_diagnostics reports it (a non-finite value or |u| > 0.5), checked every
``check`` steps.  The largest surviving Pe is found by bisection in log Pe.

    python -m paper_2504_09041_amd.stability [--scenario ma|grid|pr] [--steps N]
        [--hint previous.json]

prints one JSON object per finished point (on stderr as it goes) and one
summary object on stdout.  ``--hint`` takes the summary of an earlier run with
fewer steps: a point that failed within fewer steps also fails within more,
so its bracket starts at [pe_max / 8, pe_unstable] of that run.
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch

import workloads

from .sim import Simulation, params_from_workload


def _config(L, Ma, Pr, Pe, Ri=1.0):
    U = Ma / math.sqrt(3.0)
    cfg = workloads.config("mixed3d_64", shape=(L, L, L), U_lid=U, Pe=float(Pe), Re=float(Pe) / Pr, Ri=Ri, Pr=Pr)
    cfg["faces"][5]["u_w"] = (U, 0.0, 0.0)
    return cfg


def survives(model, L, Ma, Pr, Pe, steps, check=5000, option="A"):
    """(True, steps) if the run reaches ``steps`` with the watchdog quiet,
    else (False, step of the first failed check)."""
    cfg = _config(L, Ma, Pr, Pe)
    p = params_from_workload(cfg, "f64", model=model, thermal_option=option)
    sim = Simulation(p)
    T = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    sim.init(T)
    del T
    n = 0
    ok = True
    while n < steps:
        k = min(check, steps - n)
        sim.step(k)
        n += k
        if sim.diagnostics(4)["unstable"]:
            ok = False
            break
    sim.close()
    return ok, n


def max_stable_pe(model, L, Ma, Pr, steps, lo=10.0, hi=1e6, iters=8, log=None, check=5000):
    """Bisection in log Pe between a stable lower point and an unstable
    ``hi``.  The lower point starts at ``lo`` and is raised by factors of 3
    while the run fails there (at high Pr the small-Pe end has very large
    viscosities, which fail on their own)."""
    ok_hi, _ = survives(model, L, Ma, Pr, hi, steps, check)
    if ok_hi:
        return {"pe_max": hi, "bound": "lower (stable at the top of the range)"}
    start = lo
    while True:
        ok_lo, n_lo = survives(model, L, Ma, Pr, start, steps, check)
        if log:
            print(f"  {model} L={L} Ma={Ma} Pr={Pr} Pe={start:.4g} -> {'stable' if ok_lo else f'unstable at {n_lo}'}",
                  file=log, flush=True)
        if ok_lo:
            break
        start *= 3.0
        if start >= hi:
            return {"pe_max": None, "bound": f"no stable Pe in [{lo}, {hi})"}
    a, b = math.log(start), math.log(hi)
    for _ in range(iters):
        mid = 0.5 * (a + b)
        ok, n = survives(model, L, Ma, Pr, math.exp(mid), steps, check)
        if log:
            print(f"  {model} L={L} Ma={Ma} Pr={Pr} Pe={math.exp(mid):.4g} -> {'stable' if ok else f'unstable at {n}'}",
                  file=log, flush=True)
        if ok:
            a = mid
        else:
            b = mid
    return {"pe_max": math.exp(a), "pe_unstable": math.exp(b), "pe_low": start}


SCENARIOS = {
    # Sec. 7: (1) L = 64, Pr = 0.71, Ma swept; (2) Ma = 0.25, Pr = 0.71, L swept;
    # (3) L = 64, Ma = 0.25, Pr swept
    "ma": [(64, Ma, 0.71) for Ma in (0.01, 0.05, 0.1, 0.15, 0.2, 0.25)],
    "grid": [(L, 0.25, 0.71) for L in (32, 48, 64, 80)],
    "pr": [(64, 0.25, Pr) for Pr in (0.1, 0.71, 1.0, 2.0, 5.0)],
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--scenario", choices=tuple(SCENARIOS), action="append")
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--iters", type=int, default=7)
    ap.add_argument("--models", default="FP,MCM")
    ap.add_argument("--points", default="", help="comma list of indices into the scenario (default: all)")
    ap.add_argument("--hint", help="summary JSON of an earlier run with fewer steps (narrows the brackets)")
    ap.add_argument("--check", type=int, default=5000, help="steps between watchdog checks")
    a = ap.parse_args(argv)
    hints = {}
    if a.hint:
        with open(a.hint) as fh:
            for r in json.load(fh)["stability"]:
                if r.get("pe_max") and r.get("pe_unstable") and r.get("steps", 0) <= a.steps:
                    hints[(r["model"], r["L"], r["Ma"], r["Pr"])] = (r["pe_max"] / 8.0, r["pe_unstable"])
    if not torch.cuda.is_available():
        print("the stability study needs a GPU", file=sys.stderr)
        sys.exit(1)
    out = []
    for sc in a.scenario or ["ma"]:
        pts = SCENARIOS[sc]
        if a.points:
            pts = [pts[int(i)] for i in a.points.split(",")]
        for (L, Ma, Pr) in pts:
            for model in a.models.split(","):
                t0 = time.perf_counter()
                lo, hi = hints.get((model, L, Ma, Pr), (10.0, 1e6))
                r = max_stable_pe(model, L, Ma, Pr, a.steps, lo=lo, hi=hi, iters=a.iters, log=sys.stderr,
                                  check=a.check)
                r.update(scenario=sc, model=model, L=L, Ma=Ma, Pr=Pr, steps=a.steps,
                         seconds=time.perf_counter() - t0)
                print(json.dumps(r), file=sys.stderr, flush=True)
                out.append(r)
    print(json.dumps({"stability": out}))


if __name__ == "__main__":
    main()
