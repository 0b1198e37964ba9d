"""A second, independent route through the D2Q9 collision, for pinning the oracle.

Test helper only.  Where the oracle builds the per-node matrix C(u) from the
definition of central moments and solves C(u) f~ = kappa~, this module goes
the way Sec. 4.2 describes the transforms, written generically:

* raw moments m_pq = sum_a f_a e_ax^p e_ay^q (definition of the raw moments);
* central moments from raw ones by the binomial theorem applied to
  (e_x - u_x)^p (e_y - u_y)^q, and back with +u (the frame transform F(u) and
  its inverse, whose entries Sec. 4.2 says are the binomial coefficients);
* populations from raw moments with the printed P^-1 of App. A Step 5
  (golden fixture ``d2q9_raw_moment_matrices.json``).

The collision between them uses the paper's printed lists rather than the
oracle's generic recurrence and source rule:

* fluid attractors of Eq. D2Q9attractors (orders <= 3 fixed, the order-4
  attractor (k~20 k~02 + 2 k~11^2) / rho);
* sources of Eq. sourceCM2D, first-order moments zero, with sigma_12 taken
  with the factor 2 on its (F_y/rho) k11 term that Eq. forcing:2D gives;
* thermal option-A attractors of Eq. MvT2D;
* relaxation k~ = k + w (k^Mv - k) + (1 - w/2) sigma, second-order diagonal
  moments grouped as (k20 + k02, k20 - k02) with rates (w3, w4), orders in
  increasing sequence (App. A Step 3, App. B Step 3).
"""

from __future__ import annotations

import json
import math
import os

import torch

DT = torch.float64
EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
ORDER = ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2))
_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "d2q9_raw_moment_matrices.json")


def printed_matrices():
    """(P, P^-1) as printed in App. A Steps 1 and 5."""
    with open(_GOLDEN) as fh:
        d = json.load(fh)
    return torch.tensor(d["P"], dtype=DT), torch.tensor(d["P_inverse"], dtype=DT)


def raw_moments(f):
    """{(p, q): sum_a f_a e_ax^p e_ay^q}; f is (N, 9)."""
    return {m: sum(f[:, a] * (EX[a] ** m[0]) * (EY[a] ** m[1]) for a in range(9)) for m in ORDER}


def shift(mom, ux, uy, sign):
    """Moments about the origin shifted by sign * u: with sign = -1,
    sum_a f_a (e_x - u_x)^p (e_y - u_y)^q = sum_{i<=p, j<=q} C(p, i) C(q, j)
    (-u_x)^(p-i) (-u_y)^(q-j) m_ij; sign = +1 undoes it."""
    out = {}
    for p, q in ORDER:
        acc = 0.0 * mom[(0, 0)]
        for i in range(p + 1):
            for j in range(q + 1):
                acc = acc + (math.comb(p, i) * math.comb(q, j) * (sign * ux) ** (p - i) * (sign * uy) ** (q - j)
                             * mom[(i, j)])
        out[(p, q)] = acc
    return out


def populations(raw):
    """f = P^-1 m with the printed P^-1; returns (N, 9)."""
    _, Pinv = printed_matrices()
    m = torch.stack([raw[k] for k in ORDER], 1)
    return m @ Pinv.T


def _relax(k, mv, sig, w):
    return k + w * (mv - k) + (1.0 - 0.5 * w) * sig


def _relax_second_order(kap, mv, sig, w, out):
    """(k20 + k02, k20 - k02) relaxed at (w3, w4), then split; k11 at w5."""
    s = _relax(kap[(2, 0)] + kap[(0, 2)], mv[(2, 0)] + mv[(0, 2)], sig[(2, 0)] + sig[(0, 2)], w[3])
    d = _relax(kap[(2, 0)] - kap[(0, 2)], mv[(2, 0)] - mv[(0, 2)], sig[(2, 0)] - sig[(0, 2)], w[4])
    out[(2, 0)] = 0.5 * (s + d)
    out[(0, 2)] = 0.5 * (s - d)
    out[(1, 1)] = _relax(kap[(1, 1)], mv[(1, 1)], sig[(1, 1)], w[5])


def fluid_collide(f, F, w, cs2=1.0 / 3.0):
    """Fluid collision of (N, 9) populations under force F (N, 2) with the nine
    rates w0..w8; returns (f~, rho, u) with the half-force velocity."""
    raw = raw_moments(f)
    rho = raw[(0, 0)]
    ux = (raw[(1, 0)] + 0.5 * F[:, 0]) / rho
    uy = (raw[(0, 1)] + 0.5 * F[:, 1]) / rho
    kap = shift(raw, ux, uy, -1)
    ax, ay = F[:, 0] / rho, F[:, 1] / rho
    zero = 0.0 * rho
    sig = {(0, 0): zero, (1, 0): F[:, 0], (0, 1): F[:, 1], (2, 0): zero, (0, 2): zero, (1, 1): zero,
           (2, 1): 2 * ax * kap[(1, 1)] + ay * kap[(2, 0)],
           (1, 2): ax * kap[(0, 2)] + 2 * ay * kap[(1, 1)],
           (2, 2): 2 * (ax * kap[(1, 2)] + ay * kap[(2, 1)])}
    mv = {(0, 0): rho, (1, 0): zero, (0, 1): zero, (2, 0): cs2 * rho, (0, 2): cs2 * rho, (1, 1): zero,
          (2, 1): zero, (1, 2): zero}
    post = {}
    for slot, m in ((0, (0, 0)), (1, (1, 0)), (2, (0, 1))):
        post[m] = _relax(kap[m], mv[m], sig[m], w[slot])
    _relax_second_order(kap, mv, sig, w, post)
    for slot, m in ((6, (2, 1)), (7, (1, 2))):
        post[m] = _relax(kap[m], mv[m], sig[m], w[slot])
    mv22 = (post[(2, 0)] * post[(0, 2)] + 2 * post[(1, 1)] ** 2) / rho
    post[(2, 2)] = _relax(kap[(2, 2)], mv22, sig[(2, 2)], w[8])
    return populations(shift(post, ux, uy, +1)), rho, torch.stack([ux, uy], 1)


def thermal_collide(g, u, w, cs2T=1.0 / 3.0):
    """Thermal collision (D2Q9 thermal lattice, option A) of (N, 9) populations
    with the fluid velocity u (N, 2); returns (g~, T)."""
    raw = raw_moments(g)
    T = raw[(0, 0)]
    ux, uy = u[:, 0], u[:, 1]
    eta = shift(raw, ux, uy, -1)
    zero = 0.0 * T
    nosrc = {m: zero for m in ORDER}
    mv = {(0, 0): T, (1, 0): zero, (0, 1): zero, (2, 0): cs2T * T, (0, 2): cs2T * T, (1, 1): zero}
    post = {}
    for slot, m in ((0, (0, 0)), (1, (1, 0)), (2, (0, 1))):
        post[m] = _relax(eta[m], mv[m], zero, w[slot])
    _relax_second_order(eta, mv, nosrc, w, post)
    post[(2, 1)] = _relax(eta[(2, 1)], 2.0 / 3.0 * cs2T * post[(0, 1)], zero, w[6])
    post[(1, 2)] = _relax(eta[(1, 2)], 2.0 / 3.0 * cs2T * post[(1, 0)], zero, w[7])
    post[(2, 2)] = _relax(eta[(2, 2)], 0.5 * cs2T * (post[(2, 0)] + post[(0, 2)]), zero, w[8])
    return populations(shift(post, ux, uy, +1)), T
