"""Physics self-validation at the paper's settings.

Natural convection in the differentially heated square cavity (Sec. 6.1) and
cube (Sec. 6.2), run to a steady state on the GPU and compared with the
paper's own FPC-LBM results: Tables con1-con4 (2D, 512^2, Pr 0.71) and Table
CompareNu3D (3D, 128^3).  This checks physics, not parity: the thermal
lattice here is D2Q5 / D3Q7 (the paper's runs use D2Q9 / D3Q15), and the
characteristic velocity U0 is a parameter (the paper uses 0.01), so agreement
to a few tenths of a percent up to about one percent is the expectation.
``--paper-lattices`` runs the paper's own thermal lattices instead (D2Q9 /
D3Q15, FP64).

    python -m paper_2504_09041_amd.validate [--quick] [--paper-lattices]

prints one JSON object.  The steady state is declared when the hot-wall mean
Nusselt number changes by less than ``tol`` (relative) over one chunk of
steps.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import torch

import workloads

from .sim import Simulation, params_from_workload

# The paper's FPC-LBM values (2D: Tables con1-con4 at 512^2; 3D: Table
# CompareNu3D at 128^3).  Velocities are scaled by alpha / L; locations by L.
PAPER_2D = {
    1e3: {"nu": 1.1153, "nu_max": 1.5089, "nu_max_y": 0.0793, "nu_min": 0.6898, "nu_min_y": 0.9990,
          "u_max": 3.6418, "u_max_y": 0.8131, "v_max": 3.6900, "v_max_x": 0.1787},
    1e4: {"nu": 2.2431, "nu_max": 3.5343, "nu_min": 0.5835},
    1e5: {"nu": 4.5188, "nu_max": 7.7272, "nu_min": 0.7220},
    1e6: {"nu": 8.8116, "nu_max": 17.5230, "nu_max_y": 0.0400, "nu_min": 0.9755, "nu_min_y": 0.9990,
          "u_max": 64.8670, "u_max_y": 0.8506, "v_max": 220.5401, "v_max_x": 0.0381},
}
PAPER_3D = {1e5: {"nu": 4.3500}, 1e6: {"nu": 8.6473}}


def _alpha(p, dim):
    """Thermal diffusivity of the first-order thermal rate: c^_s^2 (1/w - 1/2)."""
    return p.cs2_T * (1.0 / p.omega_g[1] - 0.5)


def cavity(dim, Ra, n, U0=0.05, precision="f64", chunk=20000, tol=2e-6, max_steps=20_000_000, log=None,
           pair=None):
    """Run the heated cavity (hot x = 0 wall, cold x = n wall, adiabatic
    elsewhere) from the conduction profile to a steady state.  ``pair``
    overrides the lattice pair (e.g. "D2Q9-D2Q9")."""
    name = "dhc2d_64" if dim == 2 else "dhc3d_256"
    shape = (n, n, 1) if dim == 2 else (n, n, n)
    cfg = workloads.config(name, shape=shape, Ra=float(Ra), U0=float(U0), init="conduction_noise_uniform")
    if pair:
        cfg["pair"] = pair
    ref = "conduction" if precision == "f32dev" else "uniform"
    p = params_from_workload(cfg, precision, T_reference=ref)
    sim = Simulation(p)
    T_init = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    sim.init(T_init)
    del T_init
    t0 = time.perf_counter()
    nu_prev, steps, change = None, 0, float("inf")
    while steps < max_steps:
        sim.step(chunk)
        steps += chunk
        d = sim.diagnostics(0)
        if d["unstable"]:
            raise RuntimeError(f"Ra={Ra}: unstable after {steps} steps")
        nu = d["nu"]
        if nu_prev is not None:
            change = abs(nu - nu_prev) / abs(nu)
            if change < tol:
                break
        nu_prev = nu
        if log:
            print(f"  Ra={Ra:g} n={n} step={steps} Nu={nu:.6f} change={change:.2e}", file=log, flush=True)
    m = sim.macros()
    u = m["u"]
    L = n
    alpha = _alpha(p, dim)
    out = {"dim": dim, "Ra": Ra, "n": n, "U0": U0, "precision": precision, "pair": cfg["pair"], "steps": steps,
           "last_change": change, "seconds": time.perf_counter() - t0, "nu": nu}
    if dim == 2:
        # local Nusselt numbers along the hot x = 0 wall (library stencil)
        loc = sim.nusselt_local(0).reshape(-1)
        y = (torch.arange(n, device=loc.device, dtype=torch.float64) + 0.5) / L
        i_max, i_min = int(torch.argmax(loc)), int(torch.argmin(loc))
        out.update(nu_max=float(loc[i_max]), nu_max_y=float(y[i_max]), nu_min=float(loc[i_min]),
                   nu_min_y=float(y[i_min]))
        # u on the vertical centre line, v on the horizontal centre line (the
        # mid-plane lies between two node columns / rows for even n)
        ux = u[0, 0]
        uy = u[1, 0]
        uc = 0.5 * (ux[:, n // 2 - 1] + ux[:, n // 2]) if n % 2 == 0 else ux[:, n // 2]
        vc = 0.5 * (uy[n // 2 - 1, :] + uy[n // 2, :]) if n % 2 == 0 else uy[n // 2, :]
        iu, iv = int(torch.argmax(uc)), int(torch.argmax(vc))
        out.update(u_max=float(uc[iu]) * L / alpha, u_max_y=float(y[iu]), v_max=float(vc[iv]) * L / alpha,
                   v_max_x=float(y[iv]))
        ref_vals = PAPER_2D.get(float(Ra))
    else:
        ref_vals = PAPER_3D.get(float(Ra))
    if ref_vals:
        out["paper"] = ref_vals
        out["rel_diff"] = {k: (out[k] - v) / v for k, v in ref_vals.items() if k in out and not k.endswith(("_y", "_x"))}
    sim.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="2D at 128^2, Ra 1e4 only")
    ap.add_argument("--dim", type=int, default=0, help="2 or 3 (default: both)")
    ap.add_argument("--U0", type=float, default=0.05)
    ap.add_argument("--n2", type=int, default=512)
    ap.add_argument("--n3", type=int, default=128)
    ap.add_argument("--paper-lattices", action="store_true", help="D2Q9 / D3Q15 thermal lattices (FP64)")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("validation needs a GPU", file=sys.stderr)
        sys.exit(1)
    res = []
    if a.quick:
        res.append(cavity(2, 1e4, 128, U0=0.1, log=sys.stderr))
    else:
        pair2 = "D2Q9-D2Q9" if a.paper_lattices else None
        pair3 = "D3Q27-D3Q15" if a.paper_lattices else None
        if a.dim in (0, 2):
            for Ra in (1e3, 1e4, 1e5, 1e6):
                res.append(cavity(2, Ra, a.n2, U0=a.U0, log=sys.stderr, pair=pair2))
        if a.dim in (0, 3):
            for Ra in (1e5, 1e6):
                res.append(cavity(3, Ra, a.n3, U0=a.U0, precision="f64" if a.paper_lattices else "f32dev",
                                  chunk=5000, tol=5e-6, log=sys.stderr, pair=pair3))
    print(json.dumps({"validation": res}))


if __name__ == "__main__":
    main()
