"""Physics pins of the oracle's 3D fluid arithmetic and of the bulk rates (CPU).

The D3Q27 second-order rate assignment is not printed in the paper (Sec. 5.2
defers it to the authors' earlier work).  The oracle's reading relaxes the
trace k200+k020+k002 at the bulk rate (slot 7), the two deviators
k200-k020, k200-k002 (slots 8, 9) and the three off-diagonals k110, k101,
k011 (slots 4, 5, 6) at the shear rate.  These tests fix that reading by what
it implies for the continuum, so that a slot moved, a grouping row changed or
a wrong force term fails here and not only on the GPU:

* every off-diagonal shear wave u_i(x_j) decays at the viscosity of its own
  slot, nu = c_s^2 (1/w - 1/2) (the relation of Eq. transportcoeff2DFPCLBM,
  used in 3D as in 2D);
* diagonal waves (wave vector and velocity in one coordinate plane, at 45
  degrees) excite only the deviators, and decay at the deviators' viscosity in
  all three planes (isotropy of the traceless part);
* the shear decay does not depend on the trace rate at all, while a sound
  wave's damping does: Gamma = k^2/2 (2 (1 - 1/d) nu + zeta) with
  zeta = (2/d) c_s^2 (1/w_b - 1/2).  In 2D this is the bulk viscosity of
  Eq. transportcoeff2DFPCLBM (d = 2, w_b = w3); in 3D it is the same
  Chapman-Enskog result for the trace relaxed at w_b;
* with the rates of the natural-convection mapping (``oracle.params``), every
  shear wave decays at the prescribed nu;
* a uniform body force along any up axis adds exactly sum F to the momentum
  per step (Eq. forcing:3D with the half-force velocity);
* Couette flow under a moving lid on a z face and on an x face is the exact
  linear profile; a body-force-driven channel between two no-slip walls keeps
  the parabolic profile F x (H - x) / (2 nu).
"""

import math

import pytest
import torch

from oracle import sim
from oracle.collision import fluid_collide, rest_weights
from oracle.lattices import PAIRS
from oracle.params import omega_vectors
from oracle.sim import Face, Params

DT = torch.float64
P = Face("periodic", "periodic")
CS2 = 1.0 / 3.0


def _nu(w):
    return CS2 * (1.0 / w - 0.5)


def _rates3d(w4=1.0, w5=1.0, w6=1.0, w7=1.0, w8=1.0, w9=1.0):
    of = [1.0] * 27
    of[4], of[5], of[6], of[7], of[8], of[9] = w4, w5, w6, w7, w8, w9
    return of


def _params(pair, shape, omega_f, faces=None, g_beta=0.0, up=2, T0=0.0):
    lf, lg = PAIRS[pair]
    cs2T = 0.25 if lg.name == "D3Q7" else 1.0 / 3.0
    og = [1.0] * lg.Q
    for k in range(1, lg.d + 1):
        og[k] = 1.2
    return Params(pair=pair, shape=shape, omega_f=list(omega_f), omega_g=og, cs2T=cs2T, g_beta=g_beta,
                  faces=faces if faces is not None else [P] * 6, up_axis=up, T0=T0)


def _equilibrium(lf, rho, u):
    """Product-form equilibrium of density rho and velocity u (fields of the
    grid's shape), from the oracle's own collision with unit rates and no
    force: the fixed point whose central moments equal the attractors."""
    shp = rho.shape
    w = rest_weights(lf)
    uN = u.reshape(lf.d, -1).T
    f0 = w[None, :] * rho.reshape(-1, 1) * (1 + 3 * uN @ lf.E.T)
    ft, _, _ = fluid_collide(f0, torch.zeros_like(uN), lf, [1.0] * lf.Q)
    return ft.T.reshape((lf.Q,) + tuple(shp))


def _centres(shape):
    return [c.to(DT) + 0.5 for c in sim._coords(shape)]


def _fit_rate(ts, amps):
    t = torch.tensor(ts, dtype=DT)
    y = torch.log(torch.tensor(amps, dtype=DT))
    A = torch.stack([torch.ones_like(t), t], 1)
    return -float(torch.linalg.lstsq(A, y.unsqueeze(1)).solution[1, 0])


def _shear_wave_nu(omega_f, kdir, udir, n, steps):
    """Effective viscosity (fitted decay rate / k^2) of the periodic shear wave
    u = A udir sin(k kdir . x) with k = 2 pi / n, kdir . udir = 0."""
    pair = "D3Q27-D3Q7"
    lf, lg = PAIRS[pair]
    shape = tuple(n if kdir[a] else 1 for a in range(3))
    prm = _params(pair, shape, omega_f)
    co = _centres(shape)
    k = 2 * math.pi / n
    phase = sum(k * kdir[a] * co[a] for a in range(3))
    u = torch.stack([1e-3 * udir[a] * torch.sin(phase) for a in range(3)], 0)
    f = _equilibrium(lf, torch.ones_like(phase), u)
    g = torch.zeros((lg.Q,) + tuple(phase.shape), dtype=DT)
    s = torch.sin(phase)
    uu = float(sum(v * v for v in udir))
    ts, amps = [], []
    for t in range(1, steps + 1):
        f, g, mac = sim.step(prm, f, g)
        if t >= steps // 4 and t % 10 == 0:
            proj = sum(udir[a] * mac["u"][a] for a in range(3)) / uu
            ts.append(t)
            amps.append(float((proj * s).sum() / (s * s).sum()))
    return _fit_rate(ts, amps) / (k * k * sum(v * v for v in kdir))


# (wave vector direction, velocity direction, the slot whose rate sets the decay)
WAVES = {
    "ux(y)": ((0, 1, 0), (1, 0, 0), 4),
    "ux(z)": ((0, 0, 1), (1, 0, 0), 5),
    "uy(z)": ((0, 0, 1), (0, 1, 0), 6),
    "diag-xy": ((1, 1, 0), (1, -1, 0), 8),
    "diag-xz": ((1, 0, 1), (1, 0, -1), 8),
    "diag-yz": ((0, 1, 1), (0, 1, -1), 8),
}


@pytest.mark.parametrize("name", list(WAVES))
def test_shear_wave_decays_at_its_own_slot(name):
    # distinct rates on the three off-diagonal slots; the two deviators share
    # one rate (the traceless part then relaxes isotropically)
    rates = {4: 1.3, 5: 1.5, 6: 1.7, 7: 1.0, 8: 1.4, 9: 1.4}
    of = _rates3d(*(rates[k] for k in (4, 5, 6, 7, 8, 9)))
    kdir, udir, slot = WAVES[name]
    n, steps = (32, 160) if sum(kdir) == 1 else (16, 120)
    nu = _shear_wave_nu(of, kdir, udir, n, steps)
    assert abs(nu / _nu(rates[slot]) - 1) < 1e-2, (name, nu, _nu(rates[slot]))


@pytest.mark.parametrize("name", list(WAVES))
def test_natural_convection_rates_give_the_prescribed_viscosity(name):
    # the rate vector of the physical mapping (oracle.params): every shear
    # mode must see nu, whichever moments carry it
    nu_target = 0.05
    of, _, _ = omega_vectors("D3Q27-D3Q7", nu_target, nu_target / 0.71)
    kdir, udir, _ = WAVES[name]
    n, steps = (32, 160) if sum(kdir) == 1 else (16, 120)
    nu = _shear_wave_nu(of, kdir, udir, n, steps)
    assert abs(nu / nu_target - 1) < 1e-2
    assert of[7] == 1.0  # the trace (bulk) keeps the free rate 1


def test_trace_rate_leaves_shear_unchanged():
    kdir, udir, _ = WAVES["diag-xy"]
    base = _rates3d(1.4, 1.4, 1.4, 1.0, 1.4, 1.4)
    nu_b = _shear_wave_nu(base, kdir, udir, 16, steps=120)
    for w7 in (0.6, 1.8):
        nu_t = _shear_wave_nu(_rates3d(1.4, 1.4, 1.4, w7, 1.4, 1.4), kdir, udir, 16, steps=120)
        assert abs(nu_t / nu_b - 1) < 1e-8
    # the deviators do set it, and the off-diagonals do not
    nu_d = _shear_wave_nu(_rates3d(1.4, 1.4, 1.4, 1.0, 1.7, 1.7), kdir, udir, 16, steps=120)
    assert abs(nu_d / nu_b - 1) > 0.2
    nu_o = _shear_wave_nu(_rates3d(1.7, 1.7, 1.7, 1.0, 1.4, 1.4), kdir, udir, 16, steps=120)
    assert abs(nu_o / nu_b - 1) < 1e-8


def _sound_damping(pair, n, wn, wb, axis, steps):
    """Fitted amplitude damping of a right-running sound wave along ``axis``
    and the prediction k^2/2 (2 (1 - 1/d) nu + zeta), zeta = (2/d) c_s^2 (1/wb - 1/2)."""
    lf, lg = PAIRS[pair]
    d = lf.d
    of = [1.0] * lf.Q
    if d == 2:
        of[3], of[4], of[5] = wb, wn, wn
    else:
        of[7] = wb
        for k in (4, 5, 6, 8, 9):
            of[k] = wn
    shape = [1, 1, 1]
    shape[axis] = n
    shape = tuple(shape)
    prm = _params(pair, shape, of, up=1 if d == 2 else 2)
    c = _centres(shape)[axis]
    k = 2 * math.pi / n
    A, cs = 1e-4, math.sqrt(CS2)
    rho = 1 + A * torch.cos(k * c)
    u = torch.zeros((d,) + tuple(c.shape), dtype=DT)
    u[axis] = cs * A * torch.cos(k * c)
    f = _equilibrium(lf, rho, u)
    g = torch.zeros((lg.Q,) + tuple(c.shape), dtype=DT)
    cc = c.reshape(-1)
    ts, amps = [], []
    for t in range(1, steps + 1):
        f, g, mac = sim.step(prm, f, g)
        if t >= steps // 5 and t % 10 == 0:
            r = mac["rho"].reshape(-1) - 1
            v = mac["u"][axis].reshape(-1)
            a = complex(float((r * torch.cos(k * cc)).sum()), float((r * torch.sin(k * cc)).sum()))
            b = complex(float((v * torch.cos(k * cc)).sum()), float((v * torch.sin(k * cc)).sum()))
            ts.append(t)
            amps.append(abs(a + b / cs))  # the right-running component
    zeta = (2.0 / d) * CS2 * (1.0 / wb - 0.5)
    return _fit_rate(ts, amps), 0.5 * k * k * (2 * (1 - 1.0 / d) * _nu(wn) + zeta)


@pytest.mark.parametrize("pair,n,wn,wb,axis", [
    ("D2Q9-D2Q5", 48, 1.6, 1.0, 0),
    ("D2Q9-D2Q5", 48, 1.6, 1.5, 1),
    ("D3Q27-D3Q7", 32, 1.6, 1.0, 2),
    ("D3Q27-D3Q7", 32, 1.2, 0.7, 0),
])
def test_sound_wave_damping_fixes_the_bulk_rate(pair, n, wn, wb, axis):
    rate, pred = _sound_damping(pair, n, wn, wb, axis, steps=300)
    assert abs(rate / pred - 1) < 5e-3, (rate, pred)


@pytest.mark.parametrize("up", [2, 0])
def test_periodic_momentum_gain_equals_force_3d(up):
    prm = _params("D3Q27-D3Q7", (4, 3, 5), _rates3d(1.5, 1.3, 1.7, 1.0, 1.4, 1.4), g_beta=1e-3, up=up, T0=0.1)
    lf, lg = prm.lattices
    gen = torch.Generator().manual_seed(7)
    f = rest_weights(lf).reshape(-1, 1, 1, 1) * (1 + 0.02 * (torch.rand(27, 5, 3, 4, generator=gen, dtype=DT) - 0.5))
    g = rest_weights(lg, thermal=True, cs2=prm.cs2T).reshape(-1, 1, 1, 1) * (
        0.3 + 0.2 * (torch.rand(7, 5, 3, 4, generator=gen, dtype=DT) - 0.5))
    for _ in range(4):
        j0 = torch.einsum("qd,q...->d", lf.E, f)
        f, g, mac = sim.step(prm, f, g)
        j1 = torch.einsum("qd,q...->d", lf.E, f)
        F = float((prm.g_beta * (mac["T"] - prm.T0)).sum())
        assert abs(F) > 1e-4  # the force is not trivially zero
        for i in range(3):
            assert abs(float(j1[i] - j0[i]) - (F if i == up else 0.0)) < 1e-14


def test_couette_lid_on_a_z_face():
    H, U, V = 6, 0.02, -0.013
    faces = [P, P, P, P, Face("noslip", "adiabatic"), Face("lid", "adiabatic", u_w=(U, V, 0.0))]
    prm = _params("D3Q27-D3Q7", (1, 1, H), _rates3d(0.8, 0.8, 0.8, 1.0, 0.8, 0.8), faces=faces)
    f, g = sim.init_state(prm, torch.zeros(H, 1, 1, dtype=DT))
    f, g, mac = sim.run(prm, f, g, 700)
    z = torch.arange(H, dtype=DT) + 0.5
    assert torch.allclose(mac["u"][0].reshape(-1), U * z / H, atol=1e-11, rtol=0)
    assert torch.allclose(mac["u"][1].reshape(-1), V * z / H, atol=1e-11, rtol=0)
    assert mac["u"][2].abs().max() < 1e-13


def test_couette_lid_on_an_x_face():
    H, V, W = 6, -0.013, 0.02
    faces = [Face("lid", "dirichlet", T=0.0, u_w=(0.0, V, W)), Face("noslip", "dirichlet", T=0.0), P, P, P, P]
    prm = _params("D3Q27-D3Q7", (H, 1, 1), _rates3d(0.8, 0.8, 0.8, 1.0, 0.8, 0.8), faces=faces)
    f, g = sim.init_state(prm, torch.zeros(1, 1, H, dtype=DT))
    f, g, mac = sim.run(prm, f, g, 700)
    x = torch.arange(H, dtype=DT) + 0.5
    assert torch.allclose(mac["u"][1].reshape(-1), V * (H - x) / H, atol=1e-11, rtol=0)
    assert torch.allclose(mac["u"][2].reshape(-1), W * (H - x) / H, atol=1e-11, rtol=0)
    assert mac["u"][0].abs().max() < 1e-13


@pytest.mark.parametrize("wall_axis,slot", [(0, 5), (1, 6)])
def test_force_driven_channel_keeps_the_parabolic_profile(wall_axis, slot):
    # walls normal to wall_axis, force along z from a uniform temperature
    # T = 1 above T0 = 0 (adiabatic walls keep it uniform); the channel starts
    # at the exact steady profile and must stay on it
    H, gb, wn = 16, 1e-6, 1.2
    rates = {4: 1.9, 5: 1.9, 6: 1.9}
    rates[slot] = wn
    of = _rates3d(rates[4], rates[5], rates[6], 1.0, 1.5, 1.5)
    faces = [P] * 6
    faces[2 * wall_axis] = faces[2 * wall_axis + 1] = Face("noslip", "adiabatic")
    shape = [1, 1, 1]
    shape[wall_axis] = H
    shape = tuple(shape)
    prm = _params("D3Q27-D3Q7", shape, of, faces=faces, g_beta=gb, up=2, T0=0.0)
    lf, lg = prm.lattices
    s = _centres(shape)[wall_axis]
    exact = gb / (2 * _nu(wn)) * s * (H - s)
    u = torch.zeros((3,) + tuple(s.shape), dtype=DT)
    u[2] = exact
    f = _equilibrium(lf, torch.ones_like(s), u)
    g = rest_weights(lg, thermal=True, cs2=prm.cs2T).reshape(-1, 1, 1, 1) * torch.ones((1,) + tuple(s.shape),
                                                                                          dtype=DT)
    f, g, mac = sim.run(prm, f, g, 600)
    err = float((mac["u"][2] - exact).abs().max() / exact.max())
    assert err < 1e-2, err
    assert float(mac["T"].sub(1.0).abs().max()) < 1e-12
