"""Synthetic workloads: physical set-ups (pure data) and seeded input fields.

This module holds none of the method's arithmetic.  It is imported by both the
oracle-driven tests and the HIP path's callers (tests, ``bench.py``), so that
both see bit-identical inputs.  Random fields are drawn on the host in FP64
with ``numpy.random.default_rng(seed)``, except ``hashed_uniform`` (a
stateless counter-based generator for inputs too large to build on the host).

Set-ups (shapes and boundary kinds of the paper's benchmark problems,
Sec. 6.1 cavity, Sec. 6.2 cube, Sec. 7 lid-driven mixed convection, plus
Rayleigh-Benard):

* ``dhc2d_64``      - 2D differentially heated cavity, 64x64, Ra 1e4
* ``rb2d_1024x512`` - 2D Rayleigh-Benard, 1024x512, periodic in x, Ra 1e6
* ``dhc3d_256``     - 3D differentially heated cube, 256^3, Ra 1e6
* ``mixed2d_512``   - 2D lid-driven mixed convection, 512^2, Re 1e3, Ri 1
* ``rb3d_128``      - 3D Rayleigh-Benard, 128^3, periodic in x and y, Ra 1e5
* ``mixed3d_64``    - 3D lid-driven mixed convection, 64^3, D3Q15 thermal: the
                      set-up of the stability comparison of Sec. 7

Faces are listed in the order -x, +x, -y, +y, -z, +z.  In 2D the z faces are
periodic with nz = 1.
"""

from __future__ import annotations

import copy

import numpy as np

FACE_ORDER = ("-x", "+x", "-y", "+y", "-z", "+z")


def _face(fluid, thermal, T=0.0, u_w=(0.0, 0.0, 0.0)):
    return {"fluid": fluid, "thermal": thermal, "T": float(T), "u_w": tuple(float(c) for c in u_w)}


_P = _face("periodic", "periodic")

CONFIGS = {
    "dhc2d_64": {
        "pair": "D2Q9-D2Q5", "shape": (64, 64, 1), "precision": "f64",
        "flow": "natural", "Ra": 1e4, "Pr": 0.71, "U0": 0.1,
        "L_axis": 0, "up_axis": 1, "T_hot": 0.5, "T_cold": -0.5,
        "faces": [_face("noslip", "dirichlet", 0.5), _face("noslip", "dirichlet", -0.5),
                  _face("noslip", "adiabatic"), _face("noslip", "adiabatic"), _P, _P],
        "steps": 2000, "nu_face": 0, "init": "uniform_noise", "seed": 2505,
    },
    "rb2d_1024x512": {
        "pair": "D2Q9-D2Q5", "shape": (1024, 512, 1), "precision": "f64+f32dev",
        "flow": "natural", "Ra": 1e6, "Pr": 0.71, "U0": 0.05,
        "L_axis": 1, "up_axis": 1, "T_hot": 0.5, "T_cold": -0.5,
        "faces": [_P, _P, _face("noslip", "dirichlet", 0.5), _face("noslip", "dirichlet", -0.5), _P, _P],
        "steps": 50000, "nu_face": 2, "init": "rb_sinusoid", "seed": 2506,
    },
    "dhc3d_256": {
        "pair": "D3Q27-D3Q7", "shape": (256, 256, 256), "precision": "f32dev",
        "flow": "natural", "Ra": 1e6, "Pr": 0.71, "U0": 0.1,
        "L_axis": 0, "up_axis": 2, "T_hot": 0.5, "T_cold": -0.5,
        "faces": [_face("noslip", "dirichlet", 0.5), _face("noslip", "dirichlet", -0.5),
                  _face("noslip", "adiabatic"), _face("noslip", "adiabatic"),
                  _face("noslip", "adiabatic"), _face("noslip", "adiabatic")],
        "steps": 20000, "nu_face": 0, "init": "uniform_noise", "seed": 2507,
    },
    "mixed2d_512": {
        "pair": "D2Q9-D2Q5", "shape": (512, 512, 1), "precision": "f32dev",
        "flow": "mixed", "Re": 1000.0, "Ri": 1.0, "Pe": 1e3, "U_lid": 0.1,
        "L_axis": 1, "up_axis": 1, "T_hot": 0.5, "T_cold": -0.5,
        "faces": [_face("noslip", "adiabatic"), _face("noslip", "adiabatic"),
                  _face("noslip", "dirichlet", -0.5), _face("lid", "dirichlet", 0.5, (0.1, 0.0, 0.0)),
                  _P, _P],
        "steps": 10000, "nu_face": 3, "init": "conduction_noise_uniform", "seed": 2508,
        "J_window": (5000, 10000), "checkpoint_every": 100, "grad_face": 2,
    },
    # Stability comparison of Sec. 7: lid-driven cube, hot moving top, cold
    # bottom, adiabatic sides; the paper's own thermal lattice (D3Q15).  Ma
    # and Pe are swept (Re = Pe / Pr); the buoyancy strength is not given in
    # the paper and is set by Ri = 1.
    "mixed3d_64": {
        "pair": "D3Q27-D3Q15", "shape": (64, 64, 64), "precision": "f64",
        "flow": "mixed", "Re": 710.0, "Ri": 1.0, "Pe": 1e3, "U_lid": 0.25 / 3 ** 0.5, "Pr": 0.71,
        "L_axis": 2, "up_axis": 2, "T_hot": 2.0, "T_cold": 1.0,
        "faces": [_face("noslip", "adiabatic"), _face("noslip", "adiabatic"),
                  _face("noslip", "adiabatic"), _face("noslip", "adiabatic"),
                  _face("noslip", "dirichlet", 1.0), _face("lid", "dirichlet", 2.0, (0.25 / 3 ** 0.5, 0.0, 0.0))],
        "steps": 1_000_000, "nu_face": 4, "init": "conduction_noise_uniform", "seed": 2510,
    },
    "rb3d_128": {
        "pair": "D3Q27-D3Q7", "shape": (128, 128, 128), "precision": "f32dev",
        "flow": "natural", "Ra": 1e5, "Pr": 0.71, "U0": 0.1,
        "L_axis": 2, "up_axis": 2, "T_hot": 0.5, "T_cold": -0.5,
        "faces": [_P, _P, _P, _P, _face("noslip", "dirichlet", 0.5), _face("noslip", "dirichlet", -0.5)],
        "steps": 3000, "nu_face": 4, "init": "conduction_noise_gauss", "seed": 2509,
    },
}


def config(name, **override):
    """A deep copy of a named set-up with optional overrides (e.g. shape)."""
    cfg = copy.deepcopy(CONFIGS[name])
    for k, v in override.items():
        cfg[k] = v
    return cfg


def _node_centres(n):
    return np.arange(n, dtype=np.float64) + 0.5


def initial_temperature(cfg, seed=None):
    """Seeded initial temperature field, shape (nz, ny, nx), float64."""
    nx, ny, nz = cfg["shape"]
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    kind = cfg["init"]
    Th, Tc = cfg["T_hot"], cfg["T_cold"]
    if kind == "uniform_noise":
        return rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx)) + 0.5 * (Th + Tc)
    up = cfg["L_axis"]
    H = cfg["shape"][up]
    s = _node_centres(H) / H  # 0..1 along the heated axis
    # linear conduction profile between the two Dirichlet faces of that axis
    lo = cfg["faces"][2 * up]["T"]
    hi = cfg["faces"][2 * up + 1]["T"]
    prof = lo + (hi - lo) * s
    shape_b = [1, 1, 1]
    shape_b[2 - up] = H
    base = np.broadcast_to(prof.reshape(shape_b), (nz, ny, nx)).copy()
    if kind == "rb_sinusoid":
        x = _node_centres(nx)
        y = _node_centres(ny)
        pert = 1e-3 * np.cos(2 * np.pi * x / (2 * H))[None, None, :] * np.sin(np.pi * y / H)[None, :, None]
        return base + pert + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    if kind == "conduction_noise_uniform":
        return base + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    if kind == "conduction_noise_gauss":
        return base + rng.normal(0.0, 1e-3, size=(nz, ny, nx))
    raise ValueError(kind)


def uniform_field(shape, seed, lo=-1.0, hi=1.0):
    """Seeded uniform noise of any shape (e.g. population perturbations)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def unit_directions(n, count, seed0=0):
    """``count`` seeded standard-normal directions of length n, unit-normalised
    (seeds seed0 .. seed0+count-1), for finite-difference checks."""
    out = []
    for s in range(seed0, seed0 + count):
        v = np.random.default_rng(s).standard_normal(n)
        out.append(v / np.linalg.norm(v))
    return np.stack(out)


# --- counter-based noise -------------------------------------------------
# A stateless generator, so that an input of any size can be built on the GPU
# in full and re-evaluated on the CPU at sampled entries only.  The mixing
# function is the "lowbias32" integer hash (C. Wellons, hash-prospector):
#   x ^= x >> 16; x *= 0x7feb352d; x ^= x >> 15; x *= 0x846ca68b; x ^= x >> 16
# (all arithmetic modulo 2^32).  It is written here with int64 tensors and a
# 16-bit split multiply so that no intermediate overflows on any device.

_M32 = 0xFFFFFFFF


def _mulmod32(x, c):
    lo = (x & 0xFFFF) * c
    hi = (((x >> 16) * c) & 0xFFFF) << 16
    return (lo + hi) & _M32


def _lowbias32(x):
    x = x ^ (x >> 16)
    x = _mulmod32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mulmod32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def hashed_uniform(index, seed):
    """Uniform values in [-1, 1) for integer counters ``index`` (an int64
    torch tensor on any device, values < 2^32) and an integer ``seed``."""
    import torch

    s = _lowbias32(torch.full_like(index, (seed * 0x9E3779B9) & _M32))
    h = _lowbias32((index & _M32) ^ s)
    return h.to(torch.float64) * (2.0 / 4294967296.0) - 1.0
