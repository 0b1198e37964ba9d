"""Physical set-up -> lattice parameters, for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/lattices.py``).

* Natural convection (Sec. 6.1): Ra = g beta dT L^3 / (nu alpha),
  Pr = nu / alpha, and the force scale F0 = U0^2 / L = g beta dT.  Hence
  nu = U0 L sqrt(Pr / Ra), alpha = nu / Pr.
* Mixed convection (Sec. 7): Pe = U L / alpha; with Re = U L / nu and the
  Richardson number Ri = g beta dT L / U^2.
* Rates: nu = c_s^2 (1/w - 1/2) for the shear rates (Eq.
  transportcoeff2DFPCLBM, c_s^2 = 1/3); alpha = c^_s^2 (1/w - 1/2) for the
  first-order thermal rates (Eq. thermaltransportcoeff2DFPCLBM / 3D).  Every
  other rate is 1 (App. A, B, C).  The 2D bulk rate w3 is left at 1 (the
  paper never fixes the bulk viscosity).  In 3D the bulk (trace) rate is 1 and
  the two deviators and three off-diagonal second-order moments carry the
  shear rate.
* c^_s^2 defaults: 1/3 (D2Q5, D2Q9, D3Q15); 1/4 for D3Q7, where 1/3 would
  make the rest weight 1 - 3 c^_s^2 vanish.
"""

from __future__ import annotations

import math

from .lattices import PAIRS
from .sim import Face, Params

DEFAULT_CS2T = {"D2Q5": 1.0 / 3.0, "D3Q7": 0.25, "D2Q9-thermal": 1.0 / 3.0, "D3Q15-thermal": 1.0 / 3.0}


def rate_from_diffusivity(D, c2):
    return 1.0 / (D / c2 + 0.5)


def omega_vectors(pair, nu, alpha, cs2=1.0 / 3.0, cs2T=None):
    lf, lg = PAIRS[pair]
    cs2T = DEFAULT_CS2T[lg.name] if cs2T is None else cs2T
    wn = rate_from_diffusivity(nu, cs2)
    wa = rate_from_diffusivity(alpha, cs2T)
    of = [1.0] * lf.Q
    if lf.d == 2:
        of[4] = wn  # k20 - k02
        of[5] = wn  # k11
    else:
        for k in (4, 5, 6, 8, 9):  # off-diagonals and the two deviators
            of[k] = wn
    og = [1.0] * lg.Q
    for k in range(1, 1 + lg.d):
        og[k] = wa
    return of, og, cs2T


def faces_from_config(cfg):
    out = []
    for fd in cfg["faces"]:
        out.append(Face(fluid=fd["fluid"], thermal=fd["thermal"], T=float(fd.get("T", 0.0)),
                        u_w=tuple(fd.get("u_w", (0.0, 0.0, 0.0)))))
    return out


def params_from_config(cfg, shape=None, cs2T=None, model="FP", thermal_option="A", **override):
    """Lattice parameters of a workload description (``workloads.configs``)."""
    shape = tuple(cfg["shape"]) if shape is None else tuple(shape)
    L = shape[cfg["L_axis"]]
    dT = cfg["T_hot"] - cfg["T_cold"]
    if cfg["flow"] == "natural":
        U0 = cfg["U0"]
        nu = U0 * L * math.sqrt(cfg["Pr"] / cfg["Ra"])
        alpha = nu / cfg["Pr"]
        g_beta = U0 * U0 / L / dT
    elif cfg["flow"] == "mixed":
        U = cfg["U_lid"]
        nu = U * L / cfg["Re"]
        alpha = U * L / cfg["Pe"]
        g_beta = cfg["Ri"] * U * U / L / dT
    else:
        raise ValueError(cfg["flow"])
    of, og, c2t = omega_vectors(cfg["pair"], nu, alpha, cs2T=cs2T)
    prm = Params(
        pair=cfg["pair"], shape=shape, omega_f=of, omega_g=og, cs2T=c2t, g_beta=g_beta,
        T0=0.5 * (cfg["T_hot"] + cfg["T_cold"]), up_axis=cfg["up_axis"],
        faces=faces_from_config(cfg), model=model, thermal_option=thermal_option, dT_ref=dT,
    )
    for k, v in override.items():
        setattr(prm, k, v)
    return prm
