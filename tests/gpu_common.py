"""Shared helpers of the GPU tests (test infrastructure).

Inputs come from ``workloads`` (seeded) and the oracle; the HIP path is only
ever the thing under test.
"""

from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import workloads
from oracle import sim as osim
from oracle.params import params_from_config

SMALL_CASES = {
    # name: (workload, shape)
    "dhc2d": ("dhc2d_64", (8, 8, 1)),
    "rb2d": ("rb2d_1024x512", (8, 6, 1)),
    "mixed2d": ("mixed2d_512", (9, 7, 1)),
    "dhc3d": ("dhc3d_256", (6, 5, 4)),
    "rb3d": ("rb3d_128", (5, 4, 6)),
    "lid3d": ("rb3d_128", (4, 5, 6)),  # faces replaced below: moving +z lid, Dirichlet +-z
    # rows of several 64-node storage tiles with a ragged last tile: interior
    # waves (fast path), periodic-x edge waves, x-wall edge waves
    "rb2d_tiles": ("rb2d_1024x512", (200, 5, 1)),
    "dhc3d_tiles": ("dhc3d_256", (130, 4, 3)),
}


def shift_temperature(cfg, dT0):
    """The same set-up with every temperature raised by dT0 (walls, hot/cold
    levels, hence T0): keeps T away from 0 where an attractor divides by T."""
    cfg["T_hot"] += dT0
    cfg["T_cold"] += dT0
    for fd in cfg["faces"]:
        if fd["thermal"] == "dirichlet":
            fd["T"] = float(fd["T"]) + dT0
    return cfg


def with_pair(cfg, paper_thermal):
    """The same set-up on the paper's thermal lattice (D2Q9 / D3Q15) when
    paper_thermal, else unchanged."""
    if paper_thermal:
        cfg["pair"] = "D2Q9-D2Q9" if cfg["pair"].startswith("D2Q9") else "D3Q27-D3Q15"
    return cfg


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_09041_amd import _abi

    _abi.load()  # fails loudly when the library is missing


def small_config(name):
    wl, shape = SMALL_CASES[name]
    cfg = workloads.config(wl, shape=shape)
    if name == "lid3d":
        f = cfg["faces"]
        f[5] = {"fluid": "lid", "thermal": "dirichlet", "T": -0.5, "u_w": (0.05, -0.03, 0.0)}
        f[4] = {"fluid": "noslip", "thermal": "dirichlet", "T": 0.5, "u_w": (0.0, 0.0, 0.0)}
    return cfg


def initial_T(cfg, seed=None):
    return torch.tensor(workloads.initial_temperature(cfg, seed=seed))


def perturbed_state(cfg, seed, amp=1e-2, **prm_kw):
    """Oracle initial state of a set-up, each population multiplied by
    (1 + amp * U(-1, 1)) with seeded noise.  Returns (f, g) FP64 CPU."""
    prm = params_from_config(cfg, **prm_kw)
    T = initial_T(cfg)
    # a non-trivial temperature field as well
    T = T + 0.2 * torch.tensor(workloads.uniform_field(T.shape, seed + 7))
    f, g = osim.init_state(prm, T)
    pf = torch.tensor(workloads.uniform_field(tuple(f.shape), seed))
    pg = torch.tensor(workloads.uniform_field(tuple(g.shape), seed + 1))
    return f * (1 + amp * pf), g * (1 + amp * pg)


def workload_params(cfg, precision, model="FP", thermal_option="A"):
    """C parameters; precision "f64", "f32dev" (FP32 deviations with the
    library's default storage reference: the conduction profile between a
    pair of Dirichlet walls, else T0), "f32uni" (the uniform reference T0) or
    "f32cond" (the conduction profile between the Dirichlet walls of the
    workload's L axis, set explicitly)."""
    from paper_2504_09041_amd.sim import params_from_workload

    kw = dict(model=model, thermal_option=thermal_option)
    if precision == "f32cond":
        return params_from_workload(cfg, "f32dev", T_reference="conduction", **kw)
    if precision == "f32uni":
        return params_from_workload(cfg, "f32dev", T_reference="uniform", **kw)
    return params_from_workload(cfg, precision, **kw)


def make_sim(cfg, precision, wall_profiles=None, model="FP", thermal_option="A"):
    from paper_2504_09041_amd.sim import Simulation

    return Simulation(workload_params(cfg, precision, model, thermal_option), wall_profiles=wall_profiles)


def load_state(sim, f, g, step=0):
    sim.import_fp64(torch.cat([f, g], 0).cuda(), step)


def read_state(sim):
    S = sim.export_fp64().cpu()
    return S[: sim.Qf], S[sim.Qf:]


def rel_err(a, b):
    """max |a - b| / max |b| (b the reference)."""
    scale = float(b.abs().max())
    return float((a - b).abs().max()) / (scale if scale > 0 else 1.0)


def oracle_run(cfg, f, g, nsteps, wall_T=None, model="FP", thermal_option="A"):
    prm = params_from_config(cfg, model=model, thermal_option=thermal_option)
    mac = None
    for _ in range(nsteps):
        f, g, mac = osim.step(prm, f, g, wall_T)
    return f, g, mac, prm


def sample_nodes(shape, count, seed):
    """Seeded sample of node coordinates plus every corner and a band of
    nodes next to each face (x, y, z int64 CPU tensors)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    xs = list(rng.integers(0, nx, count))
    ys = list(rng.integers(0, ny, count))
    zs = list(rng.integers(0, nz, count))
    for cx in (0, nx - 1):
        for cy in (0, ny - 1):
            for cz in (0, nz - 1):
                xs.append(cx)
                ys.append(cy)
                zs.append(cz)
    m = max(8, count // 8)
    for axis, n in enumerate((nx, ny, nz)):
        for side in (0, 1, n - 2, n - 1):
            if not 0 <= side < n:
                continue
            c = [rng.integers(0, nx, m), rng.integers(0, ny, m), rng.integers(0, nz, m)]
            c[axis] = np.full(m, side)
            xs += list(c[0])
            ys += list(c[1])
            zs += list(c[2])
    return (torch.tensor(xs, dtype=torch.int64), torch.tensor(ys, dtype=torch.int64),
            torch.tensor(zs, dtype=torch.int64))


def hashed_state_getters(shape, Qf, Qg, wf, wg, seed, amp=1e-2, Tamp=0.5):
    """get_f, get_g evaluating a hashed input state at given nodes (on the
    device of the index tensors): f = w (1 + amp h), g = w^T Tamp h'."""
    nx, ny, nz = shape
    N = nx * ny * nz

    def get_f(a, z, y, x):
        idx = a * N + (z * ny + y) * nx + x
        return wf[a].item() * (1.0 + amp * workloads.hashed_uniform(idx, seed))

    def get_g(a, z, y, x):
        idx = a * N + (z * ny + y) * nx + x
        return wg[a].item() * Tamp * workloads.hashed_uniform(idx, seed + 1)

    return get_f, get_g


def full_hashed_state(shape, Qf, Qg, wf, wg, seed, device, amp=1e-2, Tamp=0.5):
    """The whole hashed state as one FP64 device tensor (Qf + Qg, nz, ny, nx)."""
    nx, ny, nz = shape
    gf, gg = hashed_state_getters(shape, Qf, Qg, wf, wg, seed, amp, Tamp)
    z, y, x = torch.meshgrid(torch.arange(nz, device=device), torch.arange(ny, device=device),
                             torch.arange(nx, device=device), indexing="ij")
    out = torch.empty((Qf + Qg, nz, ny, nx), dtype=torch.float64, device=device)
    for a in range(Qf):
        out[a] = gf(a, z, y, x)
    for a in range(Qg):
        out[Qf + a] = gg(a, z, y, x)
    return out


def finite_and_close(x, tol):
    return math.isfinite(x) and x <= tol


def pull_transpose(prm, mu_f, mu_g):
    """pull^T mu: the transpose of the oracle's streaming step (the pull with
    its wall rules, an affine map of the state, so its transpose does not
    depend on the state) applied to mu, through autograd."""
    lf, lg = prm.lattices
    Sf = torch.zeros_like(mu_f, requires_grad=True)
    Sg = torch.zeros_like(mu_g, requires_grad=True)
    pf = osim.pull(Sf, lf, prm, thermal=False)
    pg = osim.pull(Sg, lg, prm, thermal=True)
    L = (mu_f * pf).sum() + (mu_g * pg).sum()
    gf, gg = torch.autograd.grad(L, [Sf, Sg])
    return gf, gg


def adjoint_step_reference(prm, f0, g0, mu, dJdT, ke, face=None, theta=None):
    """Oracle reference of one adjoint step in the form the library carries
    the adjoint: from mu_n (adjoint of the pulled populations of step n + 1)
    and the seed of level n (weights dJdT on T_n, ke on the kinetic energy),
    mu_{n-1} = collide_n^T (pull^T mu_n + seed) at the pulled populations of
    S_{n-1} = (f0, g0), and dJ/dtheta of the Dirichlet profile theta of
    `face` (or None).  Returns (mu_{n-1} as one (Qf + Qg, ...) tensor,
    dtheta or None)."""
    Qf = f0.shape[0]
    lam_f, lam_g = pull_transpose(prm, mu[:Qf], mu[Qf:])
    lf, lg = prm.lattices
    th = theta.clone().requires_grad_(True) if theta is not None else None
    fp = osim.pull(f0, lf, prm, thermal=False)
    gp = osim.pull(g0, lg, prm, thermal=True, wall_T={face: th} if th is not None else None)
    fpl = fp.detach().requires_grad_(True)
    gpl = gp.detach().requires_grad_(True)
    fn, gn, mac = osim.collide(prm, fpl, gpl)
    L = (lam_f * fn).sum() + (lam_g * gn).sum() + (dJdT * mac["T"]).sum() + ke * osim.kinetic_energy(mac)
    mf, mg = torch.autograd.grad(L, [fpl, gpl])
    dth = torch.autograd.grad(gp, th, grad_outputs=mg)[0] if th is not None else None
    return torch.cat([mf, mg], 0), dth

