"""Node-local collision of the FP central-moment double-distribution LBM.

TEST INFRASTRUCTURE ONLY (see ``oracle/lattices.py``).  Plain FP64 on CPU,
vectorised over nodes, written from the definitions:

* central moments from their definition, kappa_k = sum_a f_a prod_d
  (e_ad - u_d)^{m_kd}  (definitions of kappa_mn after Eq. (ex)/(ey), and the
  3D analogue in Sec. 5.2), as a per-node matrix C(u);
* the back-transform by *solving* C(u) f~ = kappa~ (no hand-written inverse);
* every Markovian attractor from the generic recurrence
  (Eq. Mvcmattractor2D / Mvcmattractor3D for f, Mvcmattractor2D_g /
  Mvcmattractor3Dg for g) with the diffusion-tensor rules of
  Eq. Dij2Dselection / diffusion-tensor-parameter-3D (fluid: c_s^2 I up to
  second order, renormalised kappa~_ab / rho above) and Eq. Dij2D_goptionA /
  diffusion-tensor-parameter-3DgoptionA (thermal option A: c^_s^2 I at all
  orders) or Eq. Dij2D_g / diffusion-tensor-parameter-3Dg (option B);
* body-force sources from the three-term rule (Eq. forcing:2D / forcing:3D,
  matched to the discrete sigma of Eq. sourceCM2D and Sec. 5.2), with
  pre-collision moments and the first-order central moments taken as zero, as
  the paper does when it writes sigma_20 = 2 (F_x/rho) kappa_10 = 0;
* relaxation kappa~ = kappa + w (kappa^Mv - kappa) + (1 - w/2) sigma
  (App. A Step 3), order by order so that each higher attractor sees the
  post-collision lower moments (App. A Step 3, App. B Step 3, App. C Step 3).

The "MCM" model replaces every attractor by the Maxwellian central moment
(the same recurrence with c_s^2 I at every order fed with equilibrium lower
moments), the comparison model of Sec. 7.
"""

from __future__ import annotations

import torch

from .lattices import DT, Lattice


def _axis_powers(x, pmax):
    """[x^0, x^1, ..., x^pmax] stacked on a new last axis, by repeated products.

    Repeated products (instead of ``x ** p``) keep autograd finite at x == 0.
    """
    out = [torch.ones_like(x)]
    for _ in range(pmax):
        out.append(out[-1] * x)
    return torch.stack(out, dim=-1)


def cm_matrix(lat: Lattice, u: torch.Tensor) -> torch.Tensor:
    """C(u) with C[n, k, a] = prod_d (e_ad - u_nd)^(m_kd); u is (N, d)."""
    diff = lat.E[None, :, :] - u[:, None, :]  # (N, Q, d)
    pmax = max(max(m) for m in lat.M)
    pw = _axis_powers(diff, pmax)  # (N, Q, d, pmax+1)
    rows = []
    for m in lat.M:
        r = torch.ones_like(diff[..., 0])
        for i, p in enumerate(m):
            r = r * pw[:, :, i, p]
        rows.append(r)
    return torch.stack(rows, dim=1)  # (N, K, Q)


def raw_matrix(lat: Lattice) -> torch.Tensor:
    """P with P[k, a] = prod_d e_ad^(m_kd) (Eq. dfrm): C(0)."""
    return cm_matrix(lat, torch.zeros(1, lat.d, dtype=DT))[0]


def recurrence(m, D, lower):
    """Markovian attractor of the moment with exponents m.

    Pi^Mv_m = ( sum_i m_i (m_i - 1) D_ii Pi_{m - 2 e_i}
               + sum_{i<j} 2 m_i m_j D_ij Pi_{m - e_i - e_j} ) / |m|
    (Eq. Mvcmattractor2D in 2D; Eq. Mvcmattractor3D in 3D).  ``D[i][j]`` is the
    diffusion tensor parameter (tensors or floats); ``lower(m')`` returns the
    lower-order moment Pi_{m'}.
    """
    s = sum(m)
    d = len(m)
    acc = 0.0
    for i in range(d):
        if m[i] >= 2:
            mm = list(m)
            mm[i] -= 2
            acc = acc + m[i] * (m[i] - 1) * D[i][i] * lower(tuple(mm))
    for i in range(d):
        for j in range(i + 1, d):
            if m[i] >= 1 and m[j] >= 1:
                mm = list(m)
                mm[i] -= 1
                mm[j] -= 1
                acc = acc + 2 * m[i] * m[j] * D[i][j] * lower(tuple(mm))
    return acc / s


def _unit(d, i):
    e = [0] * d
    e[i] = 1
    return tuple(e)


def _relax_order(lat, ks, kap, Mv, sig, omega, post):
    """Relax the moments ks of one order; the diagonal second-order group (if
    the lattice has one and it lies in ks) is relaxed as its combinations."""
    grouped = ()
    if lat.combo is not None and set(lat.combo[0]) <= set(ks):
        grouped = lat.combo[0]
        R = torch.tensor(lat.combo[1], dtype=DT)
        kv = torch.stack([kap[:, k] for k in grouped], 1)
        mv = torch.stack([Mv[k] * torch.ones_like(kap[:, 0]) for k in grouped], 1)
        sv = torch.stack([sig[k] * torch.ones_like(kap[:, 0]) for k in grouped], 1)
        w = torch.tensor([omega[k] for k in grouped], dtype=DT)
        c, cm, cs = kv @ R.T, mv @ R.T, sv @ R.T
        ct = c + w * (cm - c) + (1.0 - 0.5 * w) * cs
        back = torch.linalg.solve(R, ct.T).T  # split the combinations back
        for j, k in enumerate(grouped):
            post[lat.M[k]] = back[:, j]
    for k in ks:
        if k in grouped:
            continue
        w = omega[k]
        post[lat.M[k]] = kap[:, k] + w * (Mv[k] - kap[:, k]) + (1.0 - 0.5 * w) * sig[k]


def fluid_collide(f, F, lat: Lattice, omega, cs2=1.0 / 3.0, model="FP"):
    """Collision of the hydrodynamic populations at every node.

    f: (N, Q) pre-collision populations, F: (N, d) body force.
    Returns (f~ (N, Q), rho (N,), u (N, d)), with u the half-force velocity
    rho u = sum_a f_a e_a + F/2 (App. A Step 7).
    """
    d = lat.d
    rho = f.sum(1)
    u = (f @ lat.E + 0.5 * F) / rho[:, None]
    C = cm_matrix(lat, u)
    kap = torch.einsum("nkq,nq->nk", C, f)
    zero = torch.zeros_like(rho)

    def kpre(m):
        return zero if sum(m) == 1 else kap[:, lat.index[m]]

    sig = []
    for m in lat.M:
        acc = zero
        for i in range(d):
            if m[i] > 0:
                mm = list(m)
                mm[i] -= 1
                acc = acc + m[i] * (F[:, i] / rho) * kpre(tuple(mm))
        sig.append(acc)

    post = {}
    eq = {}

    def lower_post(m):
        s = sum(m)
        return rho if s == 0 else (zero if s == 1 else post[m])

    def lower_eq(m):
        s = sum(m)
        return rho if s == 0 else (zero if s == 1 else eq[m])

    iso = [[cs2 if i == j else 0.0 for j in range(d)] for i in range(d)]
    for s in sorted(set(sum(m) for m in lat.M)):
        ks = [k for k, m in enumerate(lat.M) if sum(m) == s]
        Mv = {}
        for k in ks:
            m = lat.M[k]
            if s == 0:
                Mv[k] = rho
            elif s == 1:
                Mv[k] = zero
            elif model == "MCM":
                Mv[k] = recurrence(m, iso, lower_eq)
            elif s == 2:
                Mv[k] = recurrence(m, iso, lower_post)
            else:
                D = [[post[tuple(a + b for a, b in zip(_unit(d, i), _unit(d, j)))] / rho
                      for j in range(d)] for i in range(d)]
                Mv[k] = recurrence(m, D, lower_post)
            eq[m] = Mv[k]
        _relax_order(lat, ks, kap, Mv, sig, omega, post)

    kt = torch.stack([post[m] for m in lat.M], 1)
    ft = torch.linalg.solve(C, kt.unsqueeze(-1)).squeeze(-1)
    return ft, rho, u


def thermal_collide(g, u, lat: Lattice, omega, cs2T, option="A", model="FP"):
    """Collision of the temperature populations at every node.

    g: (N, Q) pre-collision populations, u: (N, d) fluid velocity (the same u
    as the fluid collision, App. B Step 2).  Returns (g~ (N, Q), T (N,)).
    """
    d = lat.d
    T = g.sum(1)
    C = cm_matrix(lat, u)
    eta = torch.einsum("nkq,nq->nk", C, g)
    zero = torch.zeros_like(T)
    post = {}
    eq = {}

    def lower_post(m):
        return T if sum(m) == 0 else post[m]

    def lower_eq(m):
        s = sum(m)
        return T if s == 0 else (zero if s == 1 else eq[m])

    iso = [[cs2T if i == j else 0.0 for j in range(d)] for i in range(d)]
    nosrc = [zero] * lat.Q
    for s in sorted(set(sum(m) for m in lat.M)):
        ks = [k for k, m in enumerate(lat.M) if sum(m) == s]
        Mv = {}
        for k in ks:
            m = lat.M[k]
            if s == 0:
                Mv[k] = T
            elif s == 1:
                Mv[k] = zero
            elif model == "MCM":
                Mv[k] = recurrence(m, iso, lower_eq)
            elif s == 2 or option == "A":
                Mv[k] = recurrence(m, iso, lower_post)
            else:  # option B, order > 2: renormalised by the post-collision second order
                D = [[post[tuple(a + b for a, b in zip(_unit(d, i), _unit(d, j)))] / T
                      for j in range(d)] for i in range(d)]
                Mv[k] = recurrence(m, D, lower_post)
            eq[m] = Mv[k]
        _relax_order(lat, ks, eta, Mv, nosrc, omega, post)

    et = torch.stack([post[m] for m in lat.M], 1)
    gt = torch.linalg.solve(C, et.unsqueeze(-1)).squeeze(-1)
    return gt, T


_REST_CACHE = {}


def rest_weights(lat: Lattice, thermal=False, cs2=1.0 / 3.0):
    """Populations of the rest state (density or temperature 1, u = 0, F = 0).

    Obtained as one collision with every rate equal to 1 of the uniform state
    (whose velocity is zero by symmetry): the result is the fixed point whose
    central moments equal their attractors.  These are the lattice weights.
    """
    key = (lat.name, bool(thermal), float(cs2))
    if key not in _REST_CACHE:
        x = torch.full((1, lat.Q), 1.0 / lat.Q, dtype=DT)
        ones = [1.0] * lat.Q
        if thermal:
            out, _ = thermal_collide(x, torch.zeros(1, lat.d, dtype=DT), lat, ones, cs2)
        else:
            out, _, _ = fluid_collide(x, torch.zeros(1, lat.d, dtype=DT), lat, ones, cs2)
        _REST_CACHE[key] = out[0].detach()
    return _REST_CACHE[key].clone()
