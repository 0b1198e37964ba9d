"""The paper's hand-expanded D2Q9 collision (App. A, fluid; App. B, thermal).

Used only as an independent pin of the oracle: the oracle builds C(u) from the
definition of central moments, solves for the populations and evaluates every
attractor from the generic recurrence, while this module follows the printed
Steps 1-5 term by term (raw moments, F(u), relaxation with the listed
attractors and sources, F^-1(u), P^-1).

Printed typos corrected here (each checked against the definition):
* App. A Step 2, kappa_22: the term printed "- u_x^2 2 u_y kappa'_01" is
  -2 u_x^2 u_y kappa'_01.
* App. B Step 2, eta_12: the printed "kappa'_11" is eta'_11.
* Eq. sourceCM2D, sigma_12: printed as (F_x/rho) kappa_02 + (F_y/rho) kappa_11;
  the general rule of Eq. forcing:2D gives the factor n = 2 on the second
  term, as the printed sigma_21 carries on its first.
"""

from __future__ import annotations


def raw_d2q9(f):
    """Step 1: m = P f (f is a list of 9 tensors)."""
    f0, f1, f2, f3, f4, f5, f6, f7, f8 = f
    return {
        "00": f0 + f1 + f2 + f3 + f4 + f5 + f6 + f7 + f8,
        "10": f1 - f3 + f5 - f6 - f7 + f8,
        "01": f2 - f4 + f5 + f6 - f7 - f8,
        "20": f1 + f3 + f5 + f6 + f7 + f8,
        "02": f2 + f4 + f5 + f6 + f7 + f8,
        "11": f5 - f6 + f7 - f8,
        "21": f5 + f6 - f7 - f8,
        "12": f5 - f6 - f7 + f8,
        "22": f5 + f6 + f7 + f8,
    }


def central_from_raw(r, ux, uy):
    """Step 2: m^c = F(u) m."""
    uxx, uyy = ux * ux, uy * uy
    return {
        "00": r["00"],
        "10": r["10"] - ux * r["00"],
        "01": r["01"] - uy * r["00"],
        "20": r["20"] - 2 * ux * r["10"] + uxx * r["00"],
        "02": r["02"] - 2 * uy * r["01"] + uyy * r["00"],
        "11": r["11"] - uy * r["10"] - ux * r["01"] + ux * uy * r["00"],
        "21": r["21"] - 2 * ux * r["11"] + uxx * r["01"] - uy * r["20"] + 2 * ux * uy * r["10"] - uxx * uy * r["00"],
        "12": r["12"] - 2 * uy * r["11"] + uyy * r["10"] - ux * r["02"] + 2 * ux * uy * r["01"] - ux * uyy * r["00"],
        "22": (r["22"] - 2 * ux * r["12"] + uxx * r["02"] - 2 * uy * r["21"] + 4 * ux * uy * r["11"]
               - 2 * uxx * uy * r["01"] + uyy * r["20"] - 2 * ux * uyy * r["10"] + uxx * uyy * r["00"]),
    }


def raw_from_central(k, ux, uy):
    """Step 4: m~ = F^-1(u) m~^c."""
    uxx, uyy = ux * ux, uy * uy
    return {
        "00": k["00"],
        "10": k["10"] + ux * k["00"],
        "01": k["01"] + uy * k["00"],
        "20": k["20"] + 2 * ux * k["10"] + uxx * k["00"],
        "02": k["02"] + 2 * uy * k["01"] + uyy * k["00"],
        "11": k["11"] + ux * k["01"] + uy * k["10"] + ux * uy * k["00"],
        "21": k["21"] + 2 * ux * k["11"] + uy * k["20"] + uxx * k["01"] + 2 * ux * uy * k["10"] + uxx * uy * k["00"],
        "12": k["12"] + 2 * uy * k["11"] + ux * k["02"] + 2 * ux * uy * k["01"] + uyy * k["10"] + ux * uyy * k["00"],
        "22": (k["22"] + 2 * ux * k["12"] + 2 * uy * k["21"] + 4 * ux * uy * k["11"] + uyy * k["20"]
               + uxx * k["02"] + 2 * uxx * uy * k["01"] + 2 * ux * uyy * k["10"] + uxx * uyy * k["00"]),
    }


def pops_from_raw(m):
    """Step 5: f~ = P^-1 m~."""
    return [
        m["00"] - m["20"] - m["02"] + m["22"],
        (m["10"] + m["20"] - m["12"] - m["22"]) / 2,
        (m["01"] + m["02"] - m["21"] - m["22"]) / 2,
        (-m["10"] + m["20"] + m["12"] - m["22"]) / 2,
        (-m["01"] + m["02"] + m["21"] - m["22"]) / 2,
        (m["11"] + m["21"] + m["12"] + m["22"]) / 4,
        (-m["11"] + m["21"] - m["12"] + m["22"]) / 4,
        (m["11"] - m["21"] - m["12"] + m["22"]) / 4,
        (-m["11"] - m["21"] + m["12"] + m["22"]) / 4,
    ]


def fluid_collide_appA(f, Fx, Fy, w, cs2=1.0 / 3.0):
    """App. A Steps 1-5 with the half-force velocity of Step 7.

    f: list of 9 tensors; w: the nine rates w0..w8 of App. A Step 3."""
    r = raw_d2q9(f)
    rho = r["00"]
    ux = (r["10"] + 0.5 * Fx) / rho
    uy = (r["01"] + 0.5 * Fy) / rho
    k = central_from_raw(r, ux, uy)
    # Eq. sourceCM2D: sources (first-order central moments taken as zero)
    s = {
        "00": 0.0 * rho, "10": Fx, "01": Fy, "20": 0.0 * rho, "02": 0.0 * rho, "11": 0.0 * rho,
        "21": 2 * Fx / rho * k["11"] + Fy / rho * k["20"],
        "12": Fx / rho * k["02"] + 2 * Fy / rho * k["11"],
        "22": 2 * (Fx / rho * k["12"] + Fy / rho * k["21"]),
    }
    # Eq. D2Q9attractors (orders <= 3)
    mv = {"00": rho, "10": 0.0, "01": 0.0, "20": cs2 * rho, "02": cs2 * rho, "11": 0.0, "21": 0.0, "12": 0.0}
    k2s, k2d = k["20"] + k["02"], k["20"] - k["02"]
    mv2s, mv2d = mv["20"] + mv["02"], mv["20"] - mv["02"]
    s2s, s2d = s["20"] + s["02"], s["20"] - s["02"]
    t = {}
    t["00"] = k["00"] + w[0] * (mv["00"] - k["00"]) + (1 - w[0] / 2) * s["00"]
    t["10"] = k["10"] + w[1] * (mv["10"] - k["10"]) + (1 - w[1] / 2) * s["10"]
    t["01"] = k["01"] + w[2] * (mv["01"] - k["01"]) + (1 - w[2] / 2) * s["01"]
    t2s = k2s + w[3] * (mv2s - k2s) + (1 - w[3] / 2) * s2s
    t2d = k2d + w[4] * (mv2d - k2d) + (1 - w[4] / 2) * s2d
    t["11"] = k["11"] + w[5] * (mv["11"] - k["11"]) + (1 - w[5] / 2) * s["11"]
    t["21"] = k["21"] + w[6] * (mv["21"] - k["21"]) + (1 - w[6] / 2) * s["21"]
    t["12"] = k["12"] + w[7] * (mv["12"] - k["12"]) + (1 - w[7] / 2) * s["12"]
    t["20"] = 0.5 * (t2s + t2d)
    t["02"] = 0.5 * (t2s - t2d)
    mv22 = (t["20"] * t["02"] + 2 * t["11"] * t["11"]) / rho
    t["22"] = k["22"] + w[8] * (mv22 - k["22"]) + (1 - w[8] / 2) * s["22"]
    return pops_from_raw(raw_from_central(t, ux, uy)), rho, ux, uy


def thermal_collide_appB(g, ux, uy, w, cs2T=1.0 / 3.0):
    """App. B Steps 1-5 (option A attractors, Eq. MvT2D)."""
    r = raw_d2q9(g)
    T = r["00"]
    e = central_from_raw(r, ux, uy)
    mv = {"00": T, "10": 0.0, "01": 0.0, "20": cs2T * T, "02": cs2T * T, "11": 0.0}
    t = {}
    t["00"] = e["00"] + w[0] * (mv["00"] - e["00"])
    t["10"] = e["10"] + w[1] * (mv["10"] - e["10"])
    t["01"] = e["01"] + w[2] * (mv["01"] - e["01"])
    e2s, e2d = e["20"] + e["02"], e["20"] - e["02"]
    t2s = e2s + w[3] * (mv["20"] + mv["02"] - e2s)
    t2d = e2d + w[4] * (mv["20"] - mv["02"] - e2d)
    t["11"] = e["11"] + w[5] * (mv["11"] - e["11"])
    t["20"] = 0.5 * (t2s + t2d)
    t["02"] = 0.5 * (t2s - t2d)
    mv21 = 2.0 / 3.0 * cs2T * t["01"]
    mv12 = 2.0 / 3.0 * cs2T * t["10"]
    mv22 = 0.5 * cs2T * (t["20"] + t["02"])
    t["21"] = e["21"] + w[6] * (mv21 - e["21"])
    t["12"] = e["12"] + w[7] * (mv12 - e["12"])
    t["22"] = e["22"] + w[8] * (mv22 - e["22"])
    return pops_from_raw(raw_from_central(t, ux, uy)), T
