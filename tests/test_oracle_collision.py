"""Pins of the oracle's collision (CPU only).

* the whole D2Q9 fluid / thermal collision against a second route through it
  (``tests/cm_binomial_2d.py``: binomial frame shifts, the printed P^-1, the
  printed attractor and source lists);
* the generic attractor recurrence against the attractor lists the paper
  prints for D2Q9 (Eq. D2Q9attractors, Eq. MvT2D, Eq. MvT2DoptionB), D3Q27
  (Sec. 5.2 list, with the printed kappa_122 term kappa~011 kappa~012 read as
  kappa~110 kappa~012 as in the continuous list of Eq.
  continouous-Markovian-CM-3D) and D3Q15 (Eq. g-attractorsD3Q15optionA; the
  printed eta_012 attractor lacks the factor c^_s^2 that its continuous
  counterpart carries);
* collision invariants: mass, momentum + F, temperature;
* the rest state as a fixed point;
* with every rate 1 and no force, the closed-form product equilibrium;
* FP: with unit rates above second order, the higher-order post-collision
  moments are the Gaussian (Isserlis) moments of the post-collision
  covariance, in 2D and 3D; likewise the thermal option B moments on the
  paper's D2Q9 and D3Q15 lattices.
"""

import pytest
import torch

from oracle import lattices as L
from oracle.collision import fluid_collide, recurrence, rest_weights, thermal_collide
from tests import cm_binomial_2d as B

DT = torch.float64


def _rand_state(lat, n, seed, amp=0.05, rho0=1.0):
    g = torch.Generator().manual_seed(seed)
    w = rest_weights(lat, thermal=False)
    pert = (torch.rand(n, lat.Q, generator=g, dtype=DT) - 0.5) * 2 * amp
    return rho0 * w[None, :] * (1.0 + pert)


def _rand_rates(q, seed, lo=0.6, hi=1.9):
    g = torch.Generator().manual_seed(seed)
    return [float(x) for x in lo + (hi - lo) * torch.rand(q, generator=g, dtype=DT)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fluid_collision_matches_the_binomial_route(seed):
    f = _rand_state(L.D2Q9, 64, seed)
    g = torch.Generator().manual_seed(100 + seed)
    F = (torch.rand(64, 2, generator=g, dtype=DT) - 0.5) * 1e-2
    w = _rand_rates(9, seed)
    ft, rho, u = fluid_collide(f, F, L.D2Q9, w)
    fb, rho_b, ub = B.fluid_collide(f, F, w)
    assert torch.allclose(ft, fb, atol=2e-15, rtol=0)
    assert torch.allclose(u, ub, atol=1e-16, rtol=0)


@pytest.mark.parametrize("seed", [0, 1])
def test_thermal_collision_matches_the_binomial_route(seed):
    gen = torch.Generator().manual_seed(seed)
    T = (torch.rand(64, generator=gen, dtype=DT) - 0.5)
    w9 = rest_weights(L.D2Q9_T, thermal=True)
    g9 = T[:, None] * w9[None, :] + 0.01 * (torch.rand(64, 9, generator=gen, dtype=DT) - 0.5)
    u = (torch.rand(64, 2, generator=gen, dtype=DT) - 0.5) * 0.2
    w = _rand_rates(9, 10 + seed)
    gt, _ = thermal_collide(g9, u, L.D2Q9_T, w, 1.0 / 3.0)
    gb, _ = B.thermal_collide(g9, u, w)
    assert torch.allclose(gt, gb, atol=2e-15, rtol=0)


def _lower_random(keys, seed):
    g = torch.Generator().manual_seed(seed)
    return {k: torch.rand(8, generator=g, dtype=DT) - 0.3 for k in keys}


def test_recurrence_reproduces_2d_lists():
    P = _lower_random([(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)], 3)
    rho, T = P[(0, 0)], P[(0, 0)]
    # fluid (Eq. D2Q9attractors): D' = P2 / rho above second order, first order zero
    D = [[P[(2, 0)] / rho, P[(1, 1)] / rho], [P[(1, 1)] / rho, P[(0, 2)] / rho]]
    low = lambda m: rho if sum(m) == 0 else (0.0 * rho if sum(m) == 1 else P[m])
    k22 = recurrence((2, 2), D, low)
    assert torch.allclose(k22, (P[(2, 0)] * P[(0, 2)] + 2 * P[(1, 1)] ** 2) / rho, atol=1e-15)
    assert torch.allclose(recurrence((2, 1), D, low), 0 * rho)
    # thermal option A (Eq. MvT2D)
    c = 0.3
    iso = [[c, 0.0], [0.0, c]]
    lowT = lambda m: T if sum(m) == 0 else P[m]
    assert torch.allclose(recurrence((2, 1), iso, lowT), 2 / 3 * c * P[(0, 1)], atol=1e-15)
    assert torch.allclose(recurrence((1, 2), iso, lowT), 2 / 3 * c * P[(1, 0)], atol=1e-15)
    assert torch.allclose(recurrence((2, 2), iso, lowT), 0.5 * c * (P[(2, 0)] + P[(0, 2)]), atol=1e-15)
    assert torch.allclose(recurrence((2, 0), iso, lowT), c * T, atol=1e-15)
    # thermal option B (Eq. MvT2DoptionB)
    DB = [[P[(2, 0)] / T, P[(1, 1)] / T], [P[(1, 1)] / T, P[(0, 2)] / T]]
    assert torch.allclose(recurrence((2, 1), DB, lowT),
                          2 / (3 * T) * (P[(2, 0)] * P[(0, 1)] + 2 * P[(1, 1)] * P[(1, 0)]), atol=1e-14)
    assert torch.allclose(recurrence((1, 2), DB, lowT),
                          2 / (3 * T) * (P[(0, 2)] * P[(1, 0)] + 2 * P[(1, 1)] * P[(0, 1)]), atol=1e-14)
    assert torch.allclose(recurrence((2, 2), DB, lowT),
                          (P[(2, 0)] * P[(0, 2)] + 2 * P[(1, 1)] ** 2) / T, atol=1e-14)


def test_recurrence_reproduces_d3q27_list():
    keys = [m for m in L.D3Q27.M if sum(m) in (2, 3, 4)] + [(0, 0, 0)]
    K = _lower_random(keys, 5)
    rho = K[(0, 0, 0)]

    def k(a, b, c):
        return K[(a, b, c)]

    D = [[k(2, 0, 0), k(1, 1, 0), k(1, 0, 1)], [k(1, 1, 0), k(0, 2, 0), k(0, 1, 1)], [k(1, 0, 1), k(0, 1, 1), k(0, 0, 2)]]
    D = [[x / rho for x in row] for row in D]
    low = lambda m: rho if sum(m) == 0 else (0.0 * rho if sum(m) == 1 else K[m])
    listed = {
        (2, 2, 0): (k(2, 0, 0) * k(0, 2, 0) + 2 * k(1, 1, 0) ** 2) / rho,
        (2, 0, 2): (k(2, 0, 0) * k(0, 0, 2) + 2 * k(1, 0, 1) ** 2) / rho,
        (0, 2, 2): (k(0, 2, 0) * k(0, 0, 2) + 2 * k(0, 1, 1) ** 2) / rho,
        (2, 1, 1): (k(2, 0, 0) * k(0, 1, 1) + 2 * k(1, 1, 0) * k(1, 0, 1)) / rho,
        (1, 2, 1): (k(0, 2, 0) * k(1, 0, 1) + 2 * k(1, 1, 0) * k(0, 1, 1)) / rho,
        (1, 1, 2): (k(0, 0, 2) * k(1, 1, 0) + 2 * k(0, 1, 1) * k(1, 0, 1)) / rho,
        (1, 2, 2): 2 / (5 * rho) * (k(0, 2, 0) * k(1, 0, 2) + k(0, 0, 2) * k(1, 2, 0) + 4 * k(0, 1, 1) * k(1, 1, 1)
                                    + 2 * (k(1, 0, 1) * k(0, 2, 1) + k(1, 1, 0) * k(0, 1, 2))),
        (2, 1, 2): 2 / (5 * rho) * (k(2, 0, 0) * k(0, 1, 2) + k(0, 0, 2) * k(2, 1, 0) + 4 * k(1, 0, 1) * k(1, 1, 1)
                                    + 2 * (k(1, 1, 0) * k(1, 0, 2) + k(0, 1, 1) * k(2, 0, 1))),
        (2, 2, 1): 2 / (5 * rho) * (k(2, 0, 0) * k(0, 2, 1) + k(0, 2, 0) * k(2, 0, 1) + 4 * k(1, 1, 0) * k(1, 1, 1)
                                    + 2 * (k(0, 1, 1) * k(2, 1, 0) + k(1, 0, 1) * k(1, 2, 0))),
        (2, 2, 2): 1 / (3 * rho) * (k(2, 0, 0) * k(0, 2, 2) + k(0, 2, 0) * k(2, 0, 2) + k(0, 0, 2) * k(2, 2, 0)
                                    + 4 * (k(1, 1, 0) * k(1, 1, 2) + k(1, 0, 1) * k(1, 2, 1) + k(0, 1, 1) * k(2, 1, 1))),
    }
    for m, v in listed.items():
        assert torch.allclose(recurrence(m, D, low), v, atol=1e-14), m
    for m in L.D3Q27.M:
        if sum(m) == 3:
            assert torch.allclose(recurrence(m, D, low), 0 * rho), m
    # second order with D' = c_s^2 I: c_s^2 rho on the diagonal, zero off it
    iso = [[1 / 3 if i == j else 0.0 for j in range(3)] for i in range(3)]
    assert torch.allclose(recurrence((2, 0, 0), iso, low), rho / 3)
    assert torch.allclose(recurrence((1, 1, 0), iso, low), 0 * rho)


def test_recurrence_reproduces_d3q15_thermal_list():
    keys = [m for m in L.D3Q15_T.M if sum(m) in (1, 2)] + [(0, 0, 0)]
    K = _lower_random(keys, 9)
    T = K[(0, 0, 0)]
    c = 1 / 3
    iso = [[c if i == j else 0.0 for j in range(3)] for i in range(3)]
    low = lambda m: T if sum(m) == 0 else K[m]
    assert torch.allclose(recurrence((1, 2, 0), iso, low), 2 / 3 * c * K[(1, 0, 0)])
    assert torch.allclose(recurrence((0, 1, 2), iso, low), 2 / 3 * c * K[(0, 1, 0)])
    assert torch.allclose(recurrence((2, 0, 1), iso, low), 2 / 3 * c * K[(0, 0, 1)])
    assert torch.allclose(recurrence((1, 1, 1), iso, low), 0 * T)
    assert torch.allclose(recurrence((2, 2, 0), iso, low), 0.5 * c * (K[(2, 0, 0)] + K[(0, 2, 0)]))


@pytest.mark.parametrize("lat", [L.D2Q9, L.D3Q27])
def test_fluid_invariants(lat):
    """Sum f~ = sum f; sum f~ e = sum f e + F (kappa~_1 = F/2 for any rate)."""
    f = _rand_state(lat, 40, 21)
    g = torch.Generator().manual_seed(22)
    F = (torch.rand(40, lat.d, generator=g, dtype=DT) - 0.5) * 1e-2
    w = _rand_rates(lat.Q, 23)
    ft, rho, u = fluid_collide(f, F, lat, w)
    assert torch.allclose(ft.sum(1), f.sum(1), atol=1e-14, rtol=0)
    assert torch.allclose(ft @ lat.E, f @ lat.E + F, atol=1e-14, rtol=0)


@pytest.mark.parametrize("lat,c2", [(L.D2Q5, 1 / 3), (L.D3Q7, 0.25), (L.D2Q9_T, 1 / 3), (L.D3Q15_T, 1 / 3)])
def test_thermal_invariant(lat, c2):
    g = torch.Generator().manual_seed(31)
    gp = torch.rand(40, lat.Q, generator=g, dtype=DT) - 0.3
    u = (torch.rand(40, lat.d, generator=g, dtype=DT) - 0.5) * 0.2
    gt, T = thermal_collide(gp, u, lat, _rand_rates(lat.Q, 32), c2)
    assert torch.allclose(gt.sum(1), gp.sum(1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("lat", [L.D2Q9, L.D3Q27])
def test_rest_state_fixed_point(lat):
    w = rest_weights(lat)
    f = 1.3 * w[None, :].repeat(3, 1)
    ft, _, u = fluid_collide(f, torch.zeros(3, lat.d, dtype=DT), lat, _rand_rates(lat.Q, 41))
    assert torch.allclose(ft, f, atol=1e-15, rtol=0)


def _phi(e, u, cs2=1 / 3):
    """1D factor of the product equilibrium: phi(0) = 1 - c^2 - u^2, phi(+-1) = (c^2 + u^2 +- u)/2."""
    return torch.where(torch.as_tensor(e == 0), 1 - cs2 - u * u, 0.5 * (cs2 + u * u + e * u))


@pytest.mark.parametrize("lat", [L.D2Q9, L.D3Q27])
def test_unit_rates_give_product_equilibrium(lat):
    f = _rand_state(lat, 30, 51, amp=0.2)
    ft, rho, u = fluid_collide(f, torch.zeros(30, lat.d, dtype=DT), lat, [1.0] * lat.Q)
    for a, e in enumerate(lat.vectors):
        expect = rho.clone()
        for i in range(lat.d):
            expect = expect * _phi(float(e[i]), u[:, i])
        assert torch.allclose(ft[:, a], expect, atol=1e-15, rtol=0), a


@pytest.mark.parametrize("lat,c2", [(L.D2Q5, 1 / 3), (L.D3Q7, 0.25)])
def test_unit_rates_give_advection_diffusion_equilibrium(lat, c2):
    """Thermal D2Q5/D3Q7 with all rates 1: g_0 = T(1 - d c^2 - |u|^2), g_+-i = T(c^2 + u_i^2 +- u_i)/2."""
    g = torch.Generator().manual_seed(61)
    gp = torch.rand(30, lat.Q, generator=g, dtype=DT)
    u = (torch.rand(30, lat.d, generator=g, dtype=DT) - 0.5) * 0.3
    gt, T = thermal_collide(gp, u, lat, [1.0] * lat.Q, c2)
    assert torch.allclose(gt[:, 0], T * (1 - lat.d * c2 - (u * u).sum(1)), atol=1e-15)
    for a in range(1, lat.Q):
        i = [j for j in range(lat.d) if lat.vectors[a][j] != 0][0]
        s = lat.vectors[a][i]
        assert torch.allclose(gt[:, a], T * (c2 + u[:, i] ** 2 + s * u[:, i]) / 2, atol=1e-15)


# --- the Maxwellian comparator (MCM) and the thermal lattices of the paper ---

def _central(lat, pop, u):
    """Central moments of populations pop (n, Q) at velocity u (n, d), from the
    definition sum_a pop_a prod_d (e_ad - u_d)^m_d (written out here, not the
    oracle's matrix)."""
    out = {}
    for m in lat.M:
        acc = torch.zeros(pop.shape[0], dtype=DT)
        for a, e in enumerate(lat.vectors):
            t = pop[:, a].clone()
            for i in range(lat.d):
                for _ in range(m[i]):
                    t = t * (e[i] - u[:, i])
            acc = acc + t
        out[m] = acc
    return out


def _maxwell_cm(m, dens, c2):
    """Central moment of the continuous Maxwellian truncated to the lattice:
    dens * prod_d c(m_d) with c(0) = 1, c(1) = 0, c(2) = c^2 (matching principle)."""
    v = dens.clone()
    for k in m:
        v = v * (1.0 if k == 0 else (0.0 if k == 1 else c2))
    return v


@pytest.mark.parametrize("lat", [L.D2Q9, L.D3Q27])
def test_mcm_fluid_high_orders_are_maxwellian(lat):
    """MCM: with unit rates above second order and no force, every post-
    collision central moment of order >= 3 equals the Maxwellian value, while
    the second order keeps its own (viscous) rate.  The FP model differs there
    (products of the post-collision second order), so the check discriminates."""
    f = _rand_state(lat, 25, 71, amp=0.1)
    w = [1.0] * lat.Q
    nu_slots = (4, 5) if lat.d == 2 else (4, 5, 6, 8, 9)
    for k in nu_slots:
        w[k] = 1.7
    F = torch.zeros(25, lat.d, dtype=DT)
    ft, rho, u = fluid_collide(f, F, lat, w, model="MCM")
    cm = _central(lat, ft, u)
    for m in lat.M:
        if sum(m) >= 3:
            assert torch.allclose(cm[m], _maxwell_cm(m, rho, 1 / 3), atol=1e-15, rtol=0), m
    ft_fp, _, _ = fluid_collide(f, F, lat, w, model="FP")
    top = (2, 2) if lat.d == 2 else (2, 2, 0)
    assert float((_central(lat, ft_fp, u)[top] - _maxwell_cm(top, rho, 1 / 3)).abs().max()) > 1e-6


def _gaussian_moment(axes, S):
    """E[prod_k x_axes[k]] of a centred Gaussian with covariance S (Isserlis'
    theorem: the sum over pairings of the products of covariances)."""
    if not axes:
        return torch.ones_like(S[0][0])
    if len(axes) % 2:
        return torch.zeros_like(S[0][0])
    a, rest = axes[0], axes[1:]
    acc = torch.zeros_like(S[0][0])
    for j in range(len(rest)):
        acc = acc + S[a][rest[j]] * _gaussian_moment(rest[:j] + rest[j + 1:], S)
    return acc


@pytest.mark.parametrize("lat", [L.D2Q9, L.D3Q27])
def test_fp_fluid_high_orders_are_gaussian_moments(lat):
    """FP (Sec. 4.1): the attractors above second order are the moments of the
    stationary solution of a Fokker-Planck equation with constant diffusion
    tensor D' = kappa~_2 / rho, a centred Gaussian.  With unit rates above
    second order and no force, every post-collision central moment of order
    3-6 is therefore rho times the Gaussian moment given by Isserlis' theorem
    (odd orders vanish; e.g. kappa~_220 = rho (S_xx S_yy + 2 S_xy^2) and
    kappa~_222 = rho (S_xx S_yy S_zz + 2 (S_xx S_yz^2 + S_yy S_xz^2 + S_zz S_xy^2)
    + 8 S_xy S_xz S_yz)), a closed form independent of the recurrence that the
    oracle evaluates.  The second-order rates are off 1 (the viscous slots and
    the bulk / trace slot), so the covariance is not the isotropic c_s^2 I."""
    f = _rand_state(lat, 25, 73, amp=0.1)
    w = [1.0] * lat.Q
    second = {3: 1.3, 4: 1.7, 5: 0.8} if lat.d == 2 else {4: 1.7, 5: 0.8, 6: 1.2, 7: 1.4, 8: 0.9, 9: 1.6}
    for k, v in second.items():
        w[k] = v
    F = torch.zeros(25, lat.d, dtype=DT)
    ft, rho, u = fluid_collide(f, F, lat, w, model="FP")
    cm = _central(lat, ft, u)

    def unit2(i, j):
        m = [0] * lat.d
        m[i] += 1
        m[j] += 1
        return tuple(m)

    S = [[cm[unit2(i, j)] / rho for j in range(lat.d)] for i in range(lat.d)]
    # the second order is not isotropic: the check is not the unit-rate equilibrium
    assert float((S[0][1]).abs().max()) > 1e-4
    checked = 0
    for m in lat.M:
        if sum(m) < 3:
            continue
        axes = [i for i in range(lat.d) for _ in range(m[i])]
        ref = rho * _gaussian_moment(axes, S)
        assert torch.allclose(cm[m], ref, atol=1e-15, rtol=1e-12), m
        checked += 1
    assert checked == (3 if lat.d == 2 else 17)


@pytest.mark.parametrize("lat", [L.D2Q9_T, L.D3Q15_T])
def test_thermal_option_b_high_orders_are_gaussian_moments(lat):
    """Thermal option B (Sec. 4.4, 5.4): the attractors above second order use
    D'_ab = eta~_ab / T, so with unit rates on the first order and above second
    order the post-collision moments of order >= 3 are T times the moments of a
    centred Gaussian of covariance eta~_2 / T (Isserlis' theorem: the odd
    members vanish, eta~_22 = T (S_xx S_yy + 2 S_xy^2)), on D2Q9 and on the
    D3Q15 set (120, 012, 201, 111, 220)."""
    g = torch.Generator().manual_seed(75)
    n = 25
    c2 = 0.3
    w = rest_weights(lat, thermal=True, cs2=c2)
    T0 = 1.5 + 0.2 * torch.rand(n, generator=g, dtype=DT)
    gin = T0[:, None] * w[None, :] * (1.0 + 0.2 * (torch.rand(n, lat.Q, generator=g, dtype=DT) - 0.5))
    u = (torch.rand(n, lat.d, generator=g, dtype=DT) - 0.5) * 0.1
    om = [1.0] * lat.Q
    second = [k for k, m in enumerate(lat.M) if sum(m) == 2]
    for i, k in enumerate(second):
        om[k] = 0.6 + 0.25 * i  # never 1
    gt, T = thermal_collide(gin, u, lat, om, c2, option="B", model="FP")
    cm = _central(lat, gt, u)

    def unit2(i, j):
        m = [0] * lat.d
        m[i] += 1
        m[j] += 1
        return tuple(m)

    S = [[cm[unit2(i, j)] / T for j in range(lat.d)] for i in range(lat.d)]
    assert float((S[0][1]).abs().max()) > 1e-4
    checked = 0
    for m in lat.M:
        if sum(m) < 3:
            continue
        axes = [i for i in range(lat.d) for _ in range(m[i])]
        assert torch.allclose(cm[m], T * _gaussian_moment(axes, S), atol=1e-15, rtol=1e-12), m
        checked += 1
    assert checked == (3 if lat.d == 2 else 5)


@pytest.mark.parametrize("lat", [L.D2Q9_T, L.D3Q15_T])
def test_mcm_thermal_high_orders_are_maxwellian(lat):
    """MCM on the paper's thermal lattices: orders >= 3 relax (rate 1) to the
    Maxwellian moments T prod c(m_d) with c^2 = c^_s^2."""
    g = torch.Generator().manual_seed(81)
    gp = torch.rand(25, lat.Q, generator=g, dtype=DT) + 0.2
    u = (torch.rand(25, lat.d, generator=g, dtype=DT) - 0.5) * 0.2
    w = [1.0] * lat.Q
    for k in range(1, lat.d + 1):
        w[k] = 1.4
    c2 = 1 / 3
    gt, T = thermal_collide(gp, u, lat, w, c2, model="MCM")
    cm = _central(lat, gt, u)
    for m in lat.M:
        if sum(m) >= 3:
            assert torch.allclose(cm[m], _maxwell_cm(m, T, c2), atol=1e-14, rtol=0), m


@pytest.mark.parametrize("lat", [L.D2Q9_T, L.D3Q15_T])
def test_thermal_option_a_third_order_closed_form(lat):
    """FP option A (Eq. Dij2D_goptionA): with unit rates above first order the
    third-order moments of the form (1,2,0) relax to (2/3) c^_s^2 times the
    post-collision first-order moment (1 - w) eta_(1,0,0), evaluated here from
    the input by the definition of the central moments."""
    g = torch.Generator().manual_seed(91)
    gp = torch.rand(25, lat.Q, generator=g, dtype=DT) + 0.2
    u = (torch.rand(25, lat.d, generator=g, dtype=DT) - 0.5) * 0.2
    wa = 1.35
    w = [1.0] * lat.Q
    for k in range(1, lat.d + 1):
        w[k] = wa
    c2 = 1 / 3
    gt, T = thermal_collide(gp, u, lat, w, c2, option="A")
    pre = _central(lat, gp, u)
    post = _central(lat, gt, u)
    pairs = [((2, 1), (0, 1)), ((1, 2), (1, 0))] if lat.d == 2 else \
        [((1, 2, 0), (1, 0, 0)), ((0, 1, 2), (0, 1, 0)), ((2, 0, 1), (0, 0, 1))]
    for m, low in pairs:
        assert torch.allclose(post[m], 2 / 3 * c2 * (1 - wa) * pre[low], atol=1e-13, rtol=0), m


def _marginal(lat3, lat2, axis):
    """(Q2, Q3) 0/1 matrix summing the 3D populations over the velocity
    component along ``axis`` onto the 2D lattice of the other two axes."""
    keep = [k for k in range(3) if k != axis]
    M = torch.zeros(lat2.Q, lat3.Q, dtype=DT)
    for a, v in enumerate(lat3.vectors):
        M[lat2.vectors.index(tuple(v[k] for k in keep)), a] = 1.0
    return M, keep


def _exps3(m2, keep):
    e = [0, 0, 0]
    e[keep[0]], e[keep[1]] = m2
    return tuple(e)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("model", ["FP", "MCM"])
def test_3d_collision_of_a_marginal_is_the_2d_collision(axis, model):
    """Summing the D3Q27 / D3Q7 populations over one velocity component gives a
    D2Q9 / D2Q5 distribution whose raw and central moments are the (p, q, 0)
    moments of the 3D one, whatever u and F along the summed axis.  Their
    attractors (Eq. Mvcmattractor3D restricted to one plane), sources
    (Eq. forcing:3D with one index zero) and relaxations are the 2D ones of
    Sec. 4, as long as the diagonal second-order group relaxes at one rate in
    both.  So the marginal of the 3D collision must equal the 2D collision of
    the marginal: this ties every 3D term that touches a coordinate plane to
    the 2D collision, which its own pins fix."""
    n = 40
    gen = torch.Generator().manual_seed(31 + axis)
    f3 = _rand_state(L.D3Q27, n, 40 + axis)
    F3 = (torch.rand(n, 3, generator=gen, dtype=DT) - 0.5) * 2e-2
    w3 = _rand_rates(27, 50 + axis)
    wd = 1.37
    w3[7] = w3[8] = w3[9] = wd
    M, keep = _marginal(L.D3Q27, L.D2Q9, axis)
    w2 = [w3[L.D3Q27.index[_exps3(m, keep)]] for m in L.D2Q9.M]
    w2[3] = w2[4] = wd
    ft3, rho3, u3 = fluid_collide(f3, F3, L.D3Q27, w3, model=model)
    ft2, rho2, u2 = fluid_collide(f3 @ M.T, F3[:, keep], L.D2Q9, w2, model=model)
    assert torch.allclose(ft3 @ M.T, ft2, atol=2e-15, rtol=0)
    assert torch.allclose(u3[:, keep], u2, atol=1e-16, rtol=0)
    # thermal: D3Q7 onto D2Q5 with the same c^_s^2 and rates
    c2 = 0.25
    T = 0.3 + 0.1 * torch.rand(n, generator=gen, dtype=DT)
    g3 = T[:, None] * rest_weights(L.D3Q7, thermal=True, cs2=c2)[None, :] + 0.01 * (
        torch.rand(n, 7, generator=gen, dtype=DT) - 0.5)
    wg3 = _rand_rates(7, 60 + axis)
    wg3[4] = wg3[5] = wg3[6] = wd
    Mg, _ = _marginal(L.D3Q7, L.D2Q5, axis)
    wg2 = [1.0, wg3[1 + keep[0]], wg3[1 + keep[1]], wd, wd]
    gt3, _ = thermal_collide(g3, u3, L.D3Q7, wg3, c2, model=model)
    gt2, _ = thermal_collide(g3 @ Mg.T, u3[:, keep], L.D2Q5, wg2, c2, model=model)
    assert torch.allclose(gt3 @ Mg.T, gt2, atol=2e-15, rtol=0)
