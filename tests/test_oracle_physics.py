"""Physics pins of the oracle's streaming, walls, coupling and diagnostics (CPU).

* conservation: periodic box (mass, momentum, sum T; with gravity the momentum
  grows by sum F per step); closed box with adiabatic no-slip walls (mass and
  sum T);
* transport coefficients: a shear wave decays as exp(-nu k^2 t) with
  nu = c_s^2 (1/w - 1/2), a temperature mode as exp(-alpha k^2 t) with
  alpha = c^_s^2 (1/w - 1/2); an advected mode moves at the imposed velocity;
* walls: Couette flow under a moving lid reaches the exact linear profile;
  conduction between two Dirichlet walls reaches the linear profile with
  Nu = 1 on the hot wall and -1 on the cold one;
* the wall-gradient stencil is exact for quadratic profiles;
* coupling: Rayleigh-Benard with Lx = 2H is stable below the rigid-rigid
  onset (Ra_c ~ 1708) and unstable above it; a cavity at Ra = 10 stays at
  Nu ~ 1.
"""

import math

import pytest
import torch

from oracle import sim
from oracle.collision import fluid_collide, rest_weights
from oracle.lattices import PAIRS
from oracle.params import rate_from_diffusivity
from oracle.sim import Face, Params

DT = torch.float64
P = Face("periodic", "periodic")


def _params(pair, shape, faces, wn=1.5, wa=1.4, g_beta=0.0, cs2T=None, up=1):
    lf, lg = PAIRS[pair]
    cs2T = (0.25 if lg.name == "D3Q7" else 1 / 3) if cs2T is None else cs2T
    of = [1.0] * lf.Q
    if lf.d == 2:
        of[4] = of[5] = wn
    else:
        for k in (4, 5, 6, 8, 9):
            of[k] = wn
    og = [1.0] * lg.Q
    for k in range(1, lg.d + 1):
        og[k] = wa
    return Params(pair=pair, shape=shape, omega_f=of, omega_g=og, cs2T=cs2T, g_beta=g_beta,
                  faces=faces, up_axis=up)


def _random_state(prm, seed, amp=0.02):
    lf, lg = prm.lattices
    nx, ny, nz = prm.shape
    gen = torch.Generator().manual_seed(seed)
    wf = rest_weights(lf)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    f = wf.reshape(-1, 1, 1, 1) * (1 + amp * (torch.rand(lf.Q, nz, ny, nx, generator=gen, dtype=DT) - 0.5))
    g = wg.reshape(-1, 1, 1, 1) * (0.3 + amp * (torch.rand(lg.Q, nz, ny, nx, generator=gen, dtype=DT) - 0.5))
    return f, g


def _equilibrium_fluid(lf, u):
    """Product equilibrium at density 1 and velocity field u (d, nz, ny, nx),
    obtained from the oracle's own collision with unit rates and no force."""
    shp = u.shape[1:]
    w = rest_weights(lf)
    uN = u.reshape(lf.d, -1).T
    f0 = w[None, :] * (1 + 3 * uN @ lf.E.T)
    ft, _, _ = fluid_collide(f0, torch.zeros_like(uN), lf, [1.0] * lf.Q)
    return ft.T.reshape((lf.Q,) + tuple(shp))


@pytest.mark.parametrize("pair,shape", [("D2Q9-D2Q5", (8, 6, 1)), ("D3Q27-D3Q7", (4, 5, 3)),
                                        ("D2Q9-D2Q9", (7, 6, 1)), ("D3Q27-D3Q15", (4, 3, 5))])
def test_periodic_conservation(pair, shape):
    prm = _params(pair, shape, [P] * 6)
    f, g = _random_state(prm, 1)
    lf = prm.lattices[0]
    m0, j0, t0 = f.sum(), torch.einsum("qd,q...->d", lf.E, f), g.sum()
    f, g, _ = sim.run(prm, f, g, 60)
    assert abs(float(f.sum() - m0)) < 1e-11 * float(m0)
    assert torch.allclose(torch.einsum("qd,q...->d", lf.E, f), j0, atol=1e-12)
    assert abs(float(g.sum() - t0)) < 1e-12 * float(abs(t0))


def test_periodic_momentum_gain_equals_force():
    prm = _params("D2Q9-D2Q5", (6, 5, 1), [P] * 6, g_beta=1e-3)
    f, g = _random_state(prm, 2)
    lf = prm.lattices[0]
    for _ in range(5):
        j0 = torch.einsum("qd,q...->d", lf.E, f)
        f, g, mac = sim.step(prm, f, g)
        j1 = torch.einsum("qd,q...->d", lf.E, f)
        Fy = (prm.g_beta * (mac["T"] - prm.T0)).sum()
        assert abs(float(j1[0] - j0[0])) < 1e-14
        assert abs(float(j1[1] - j0[1] - Fy)) < 1e-14


@pytest.mark.parametrize("pair,shape", [("D2Q9-D2Q5", (7, 6, 1)), ("D3Q27-D3Q7", (4, 4, 3)),
                                        ("D2Q9-D2Q9", (6, 7, 1)), ("D3Q27-D3Q15", (4, 3, 4))])
def test_closed_box_conservation(pair, shape):
    wall = Face("noslip", "adiabatic")
    faces = [wall] * 4 + ([P, P] if shape[2] == 1 else [wall, wall])
    prm = _params(pair, shape, faces, g_beta=2e-4, up=1 if shape[2] == 1 else 2)
    f, g = _random_state(prm, 3)
    m0, t0 = f.sum(), g.sum()
    f, g, _ = sim.run(prm, f, g, 60)
    assert abs(float(f.sum() - m0)) < 1e-12 * float(m0)
    assert abs(float(g.sum() - t0)) < 1e-12 * float(abs(t0))


def _fit_rate(ts, amps):
    t = torch.tensor(ts, dtype=DT)
    y = torch.log(torch.tensor(amps, dtype=DT))
    A = torch.stack([torch.ones_like(t), t], 1)
    sol = torch.linalg.lstsq(A, y.unsqueeze(1)).solution
    return -float(sol[1, 0])


@pytest.mark.parametrize("diagonal", [False, True])
def test_shear_wave_decay(diagonal):
    wn = 1.6
    nu = (1 / wn - 0.5) / 3
    if diagonal:
        n = 32
        shape = (n, n, 1)
        kv = (2 * math.pi / n, 2 * math.pi / n)
    else:
        n = 64
        shape = (1, n, 1)
        kv = (0.0, 2 * math.pi / n)
    prm = _params("D2Q9-D2Q5", shape, [P] * 6, wn=wn)
    lf = prm.lattices[0]
    x, y, _ = sim._coords(shape)
    x = x.to(DT) + 0.5
    y = y.to(DT) + 0.5
    phase = kv[0] * x + kv[1] * y
    A0 = 1e-3
    if diagonal:
        u = torch.stack([A0 * torch.sin(phase), -A0 * torch.sin(phase)], 0)
    else:
        u = torch.stack([A0 * torch.sin(phase), 0 * phase], 0)
    f = _equilibrium_fluid(lf, u)
    g = rest_weights(prm.lattices[1], thermal=True).reshape(-1, 1, 1, 1).expand(5, *f.shape[1:]).clone()
    ts, amps = [], []
    for t in range(1, 401):
        f, g, mac = sim.step(prm, f, g)
        if t >= 100 and t % 25 == 0:
            ts.append(t)
            amps.append(float((mac["u"][0] * torch.sin(phase)).sum() / (torch.sin(phase) ** 2).sum()))
    k2 = kv[0] ** 2 + kv[1] ** 2
    rate = _fit_rate(ts, amps)
    assert abs(rate / (nu * k2) - 1) < 1e-2


@pytest.mark.parametrize("pair,shape,axis", [("D2Q9-D2Q5", (64, 1, 1), 0), ("D3Q27-D3Q7", (1, 1, 48), 2),
                                             ("D2Q9-D2Q9", (1, 64, 1), 1), ("D3Q27-D3Q15", (48, 1, 1), 0)])
@pytest.mark.parametrize("u0", [0.0, 0.05])
def test_thermal_mode_decay_and_advection(pair, shape, axis, u0):
    wa = 1.3
    prm = _params(pair, shape, [P] * 6, wa=wa)
    lf, lg = prm.lattices
    alpha = prm.cs2T * (1 / wa - 0.5)
    n = shape[axis]
    k = 2 * math.pi / n
    c = sim._coords(shape)[axis].to(DT) + 0.5
    uvec = torch.zeros((lf.d,) + tuple(c.shape), dtype=DT)
    uvec[axis if lf.d == 3 else axis] = u0
    f = _equilibrium_fluid(lf, uvec)
    T = 1e-3 * torch.sin(k * c)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    g = wg.reshape(-1, 1, 1, 1) * T.unsqueeze(0)
    ts, amps, phases = [], [], []
    for t in range(1, 301):
        f, g, mac = sim.step(prm, f, g)
        if t >= 60 and t % 20 == 0:
            Tn = mac["T"]
            a_s = float((Tn * torch.sin(k * c)).sum() / (torch.sin(k * c) ** 2).sum())
            a_c = float((Tn * torch.cos(k * c)).sum() / (torch.cos(k * c) ** 2).sum())
            ts.append(t)
            amps.append(math.hypot(a_s, a_c))
            phases.append(math.atan2(-a_c, a_s))
    rate = _fit_rate(ts, amps)
    assert abs(rate / (alpha * k * k) - 1) < 1e-2
    if u0 > 0:
        speed = (phases[-1] - phases[0]) / (ts[-1] - ts[0]) / k
        assert abs(speed / u0 - 1) < 1e-2


def test_couette_lid_linear_profile():
    H, U = 8, 0.02
    faces = [P, P, Face("noslip", "adiabatic"), Face("lid", "adiabatic", u_w=(U, 0.0, 0.0)), P, P]
    prm = _params("D2Q9-D2Q5", (1, H, 1), faces, wn=0.8)
    T = torch.zeros(1, H, 1, dtype=DT)
    f, g = sim.init_state(prm, T)
    f, g, mac = sim.run(prm, f, g, 2000)
    y = torch.arange(H, dtype=DT) + 0.5
    assert torch.allclose(mac["u"][0][0, :, 0], U * y / H, atol=1e-12, rtol=0)
    assert mac["u"][1].abs().max() < 1e-13


@pytest.mark.parametrize("pair,shape,axis", [("D2Q9-D2Q5", (1, 6, 1), 1), ("D3Q27-D3Q7", (1, 1, 6), 2),
                                             ("D2Q9-D2Q9", (1, 6, 1), 1), ("D3Q27-D3Q15", (1, 1, 6), 2)])
def test_conduction_profile_and_nusselt(pair, shape, axis):
    faces = [P] * 6
    faces[2 * axis] = Face("noslip", "dirichlet", T=0.5)
    faces[2 * axis + 1] = Face("noslip", "dirichlet", T=-0.5)
    prm = _params(pair, shape, faces, wa=1.0, g_beta=0.0, up=axis)
    T = torch.zeros(shape[::-1], dtype=DT)
    f, g = sim.init_state(prm, T)
    f, g, mac = sim.run(prm, f, g, 900)
    H = shape[axis]
    s = torch.arange(H, dtype=DT) + 0.5
    prof = mac["T"].reshape(-1)
    assert torch.allclose(prof, 0.5 - s / H, atol=1e-11, rtol=0)
    assert abs(float(sim.nusselt(prm, mac["T"], 2 * axis)) - 1.0) < 1e-9
    assert abs(float(sim.nusselt(prm, mac["T"], 2 * axis + 1)) + 1.0) < 1e-9


def test_nusselt_stencil_exact_for_quadratics():
    prm = _params("D2Q9-D2Q5", (5, 12, 1), [P, P, Face("noslip", "dirichlet", T=0.7), Face("noslip", "dirichlet", T=0.0), P, P])
    a, b = -0.37, 0.021
    s = torch.arange(12, dtype=DT) + 0.5
    T = (0.7 + a * s + b * s * s).reshape(1, 12, 1).expand(1, 12, 5)
    nu = float(sim.nusselt(prm, T, 2))
    assert abs(nu - (-(12 / prm.dT_ref) * a)) < 1e-13


def _rb_params(Ra, H=16, U0=0.1, Pr=0.71):
    nu = U0 * H * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    faces = [P, P, Face("noslip", "dirichlet", T=0.5), Face("noslip", "dirichlet", T=-0.5), P, P]
    return _params("D2Q9-D2Q5", (2 * H, H, 1), faces, wn=rate_from_diffusivity(nu, 1 / 3),
                   wa=rate_from_diffusivity(alpha, 1 / 3), g_beta=U0 * U0 / H)


@pytest.mark.slow
def test_rayleigh_benard_onset():
    ke = {}
    for Ra in (1000.0, 3000.0):
        prm = _rb_params(Ra)
        nx, ny, _ = prm.shape
        x, y, _ = sim._coords(prm.shape)
        xs, ys = x.to(DT) + 0.5, y.to(DT) + 0.5
        T = 0.5 - ys / ny + 1e-3 * torch.cos(2 * math.pi * xs / nx) * torch.sin(math.pi * ys / ny)
        f, g = sim.init_state(prm, T)
        vals = []
        for t in range(1, 1601):
            f, g, mac = sim.step(prm, f, g)
            if t in (600, 1600):
                vals.append(float(sim.kinetic_energy(mac)))
        ke[Ra] = vals
        if Ra == 1000.0:
            assert abs(float(sim.nusselt(prm, mac["T"], 2)) - 1.0) < 1e-3
    assert ke[1000.0][1] < 0.7 * ke[1000.0][0]
    assert ke[3000.0][1] > 2.0 * ke[3000.0][0]


@pytest.mark.slow
def test_cavity_low_rayleigh_nusselt_one():
    H, U0, Pr, Ra = 16, 0.1, 0.71, 10.0
    nu = U0 * H * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    faces = [Face("noslip", "dirichlet", T=0.5), Face("noslip", "dirichlet", T=-0.5),
             Face("noslip", "adiabatic"), Face("noslip", "adiabatic"), P, P]
    prm = _params("D2Q9-D2Q5", (H, H, 1), faces, wn=rate_from_diffusivity(nu, 1 / 3),
                  wa=rate_from_diffusivity(alpha, 1 / 3), g_beta=U0 * U0 / H)
    f, g = sim.init_state(prm, torch.zeros(1, H, H, dtype=DT))
    f, g, mac = sim.run(prm, f, g, 1500)
    assert abs(float(sim.nusselt(prm, mac["T"], 0)) - 1.0) < 2e-3
    assert abs(float(sim.nusselt(prm, mac["T"], 1)) + 1.0) < 2e-3
