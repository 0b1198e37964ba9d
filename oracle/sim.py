"""Time stepping, boundaries and diagnostics of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/lattices.py``).

One time step n (the paper's loop of App. A Steps 3 -> 6 -> 7 and App. B,
written as pull-stream then collide):

1. pull: f_a(x) = f~_a(x - e_a) from the stored post-collision state S_{n-1}
   (Eq. LBMsteps-stream / LBMsteps-streamg), or a wall rule when x - e_a lies
   outside a non-periodic face;
2. macros: T = sum g, rho = sum f, F = g beta (T - T0) e_up (Boussinesq force
   of Sec. 6.1, with no density factor), u = (sum f e + F/2) / rho;
3. fluid and thermal collisions (``oracle.collision``);
4. S_n = (f~, g~).

Wall rules (the paper only names them, Sec. 6.1, and cites a textbook; these
are the standard halfway forms):

* static no-slip:   f_a(x) = f~_abar(x)
* moving wall u_w:  f_a(x) = f~_abar(x) + 2 w_a rho_w (e_a . u_w) / c_s^2,
  with rho_w = 1; a diagonal link whose source lies outside two faces uses
  the static rule;
* adiabatic:        g_a(x) = g~_abar(x)
* Dirichlet T_w:    g_a(x) = -g~_abar(x) + 2 w^T_a T_w
  (for thermal links crossing several faces: the Dirichlet rule with the mean
  of the crossed Dirichlet temperatures if any face is Dirichlet, else the
  adiabatic rule).

The weights w_a, w^T_a are the rest-state populations (``rest_weights``).

Grid: node (i, j, k) sits at (i + 1/2, j + 1/2, k + 1/2); walls lie halfway,
at 0 and n along non-periodic axes (Sec. 6.1: first fluid node at 1/2).
Arrays are stored [q][z][y][x].

Initialisation: pre-collision f = w rho0, g = w^T T_init(x); the initial state
S_0 is their collision (with F from T_init).

Diagnostics use the macros of time n (from the pulled state, Step 7).  Wall
Nusselt number (Sec. 6.1): dT/dn = -8/3 T_w + 3 T(1/2) - 1/3 T(3/2) along the
inward normal; Nu = -(L / dT_ref) dT/dn, positive for heat flowing into the
fluid (the printed definition drops this sign); <Nu> is the mean over the
wall nodes.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from .collision import fluid_collide, rest_weights, thermal_collide
from .lattices import DT, PAIRS

FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")


@dataclasses.dataclass
class Face:
    fluid: str = "noslip"  # "periodic" | "noslip" | "lid"
    thermal: str = "adiabatic"  # "periodic" | "adiabatic" | "dirichlet"
    T: float = 0.0
    u_w: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Params:
    pair: str
    shape: tuple  # (nx, ny, nz); nz = 1 in 2D
    omega_f: list
    omega_g: list
    cs2T: float
    g_beta: float
    T0: float = 0.0
    up_axis: int = 1
    faces: list = None  # 6 Face objects: -x, +x, -y, +y, -z, +z
    cs2: float = 1.0 / 3.0
    rho0: float = 1.0
    model: str = "FP"
    thermal_option: str = "A"
    dT_ref: float = 1.0

    @property
    def lattices(self):
        return PAIRS[self.pair]

    def periodic(self, axis):
        return self.faces[2 * axis].fluid == "periodic"


def _coords(shape):
    nx, ny, nz = shape
    z, y, x = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
    return (x, y, z)


def _profile_value(face_idx, prof, coords):
    """Per-node value of a wall profile on face ``face_idx``.

    A profile on a face normal to axis k is indexed by the node coordinates
    along the remaining axes, slowest first (z, y, x order without axis k)."""
    k = face_idx // 2
    other = [a for a in (2, 1, 0) if a != k]
    idx = tuple(coords[a] for a in other)
    p = prof
    if p.dim() < len(other):
        p = p.reshape((1,) * (len(other) - p.dim()) + tuple(p.shape))
    return p[idx]


def pull_at(get, lat, prm: Params, thermal: bool, coords, wall_T=None):
    """Incoming populations at the nodes ``coords`` = (x, y, z) (integer tensors
    of one shape), read through ``get(a, z, y, x)`` which returns the stored
    post-collision population a at those nodes.  Returns (Q,) + coords shape."""
    nx, ny, nz = prm.shape
    n = (nx, ny, nz)
    w = rest_weights(lat, thermal=thermal, cs2=prm.cs2T if thermal else prm.cs2)
    out = []
    for a in range(lat.Q):
        e = list(lat.vectors[a]) + [0] * (3 - lat.d)
        src = []
        crossed = []
        for k in range(3):
            s = coords[k] - e[k]
            if prm.periodic(k):
                s = torch.remainder(s, n[k])
            else:
                crossed.append((2 * k, s < 0))
                crossed.append((2 * k + 1, s >= n[k]))
                s = s.clamp(0, n[k] - 1)
            src.append(s)
        val = get(a, src[2], src[1], src[0])
        if not crossed:
            out.append(val)
            continue
        ncross = sum(m.to(torch.int64) for _, m in crossed)
        bb = get(lat.opp[a], coords[2], coords[1], coords[0])
        if not thermal:
            wall_val = bb
            for fi, m in crossed:
                face = prm.faces[fi]
                if face.fluid == "lid":
                    eu = sum(e[k] * face.u_w[k] for k in range(3))
                    add = 2.0 * w[a] * prm.rho0 * eu / prm.cs2
                    wall_val = wall_val + torch.where(m & (ncross == 1), add, 0.0)
        else:
            ndir = torch.zeros_like(val)
            tsum = torch.zeros_like(val)
            for fi, m in crossed:
                face = prm.faces[fi]
                if face.thermal == "dirichlet":
                    if wall_T is not None and wall_T.get(fi) is not None:
                        tw = _profile_value(fi, wall_T[fi], coords)
                    else:
                        tw = torch.full_like(val, face.T)
                    ndir = ndir + m.to(DT)
                    tsum = tsum + torch.where(m, tw, 0.0)
            tw_mean = tsum / torch.clamp(ndir, min=1.0)
            wall_val = torch.where(ndir > 0, -bb + 2.0 * w[a] * tw_mean, bb)
        out.append(torch.where(ncross > 0, wall_val, val))
    return torch.stack(out, 0)


def pull(S, lat, prm: Params, thermal: bool, wall_T=None):
    """Pull-stream one distribution with the wall rules; S is (Q, nz, ny, nx)."""
    return pull_at(lambda a, z, y, x: S[a][z, y, x], lat, prm, thermal, _coords(prm.shape), wall_T)


def step_at(prm: Params, get_f, get_g, coords, wall_T=None):
    """The time step evaluated only at the nodes ``coords``: (f~, g~, macros),
    each with the shape of ``coords`` after the population axis."""
    lf, lg = prm.lattices
    fp = pull_at(get_f, lf, prm, False, coords)
    gp = pull_at(get_g, lg, prm, True, coords, wall_T)
    return collide(prm, fp, gp)


def _force(prm: Params, T):
    lf = prm.lattices[0]
    Fup = prm.g_beta * (T - prm.T0)
    cols = [Fup if i == prm.up_axis else torch.zeros_like(T) for i in range(lf.d)]
    return torch.stack(cols, 1)


def collide(prm: Params, f, g):
    """Collide full fields f (Qf, nz, ny, nx), g (Qg, ...); returns (f~, g~, macros)."""
    lf, lg = prm.lattices
    shp = f.shape[1:]
    fN = f.reshape(lf.Q, -1).T
    gN = g.reshape(lg.Q, -1).T
    T = gN.sum(1)
    F = _force(prm, T)
    ft, rho, u = fluid_collide(fN, F, lf, prm.omega_f, prm.cs2, model=prm.model)
    gt, _ = thermal_collide(gN, u, lg, prm.omega_g, prm.cs2T, option=prm.thermal_option, model=prm.model)
    mac = {
        "rho": rho.reshape(shp),
        "u": u.T.reshape((lf.d,) + tuple(shp)),
        "T": T.reshape(shp),
    }
    return ft.T.reshape(f.shape), gt.T.reshape(g.shape), mac


def init_state(prm: Params, T_init):
    """S_0: the collision of f = w rho0, g = w^T T_init (T_init is (nz, ny, nx))."""
    lf, lg = prm.lattices
    wf = rest_weights(lf, thermal=False, cs2=prm.cs2)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    shp = tuple(T_init.shape)
    f = (wf * prm.rho0).reshape(-1, 1, 1, 1).expand((lf.Q,) + shp).clone()
    g = wg.reshape(-1, 1, 1, 1) * T_init.unsqueeze(0)
    ft, gt, _ = collide(prm, f, g)
    return ft, gt


def step(prm: Params, f, g, wall_T=None):
    """One time step: returns (f~_n, g~_n, macros of time n)."""
    lf, lg = prm.lattices
    fp = pull(f, lf, prm, thermal=False)
    gp = pull(g, lg, prm, thermal=True, wall_T=wall_T)
    return collide(prm, fp, gp)


def run(prm: Params, f, g, nsteps, wall_T=None):
    mac = None
    for _ in range(nsteps):
        f, g, mac = step(prm, f, g, wall_T)
    return f, g, mac


def nusselt(prm: Params, T, face_idx, wall_T=None):
    """<Nu> on one face from the time-n temperature T (nz, ny, nx)."""
    k = face_idx // 2
    n = prm.shape[k]
    dim = 2 - k  # tensor dim of axis k in (z, y, x)
    if face_idx % 2 == 0:
        T1, T2 = T.select(dim, 0), T.select(dim, 1)
    else:
        T1, T2 = T.select(dim, n - 1), T.select(dim, n - 2)
    if wall_T is not None and wall_T.get(face_idx) is not None:
        Tw = wall_T[face_idx].reshape(T1.shape)
    else:
        Tw = torch.full_like(T1, prm.faces[face_idx].T)
    dTdn = -8.0 / 3.0 * Tw + 3.0 * T1 - T2 / 3.0
    nu = -(n / prm.dT_ref) * dTdn
    return nu.mean()


def kinetic_energy(mac):
    return 0.5 * (mac["rho"] * (mac["u"] ** 2).sum(0)).sum()


def macros_of_state(prm: Params, f, g):
    """Macros recovered from a post-collision state S_n (same values as the
    time-n macros, by conservation of rho, T and kappa~_1 = F/2)."""
    lf, lg = prm.lattices
    rho = f.sum(0)
    T = g.sum(0)
    j = torch.einsum("qd,q...->d...", lf.E, f)
    Fup = prm.g_beta * (T - prm.T0)
    u = torch.stack([(j[i] - (0.5 * Fup if i == prm.up_axis else 0.0)) / rho for i in range(lf.d)], 0)
    return {"rho": rho, "u": u, "T": T}
