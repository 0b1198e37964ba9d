"""The hand-written adjoint on the paper's thermal lattices, D2Q9 (Sec. 4.4,
App. B) and D3Q15 (Sec. 5.4, App. C), through the C ABI, against the
oracle's autograd gradients.

The D2Q9 thermal moments are the tensor-product central moments (the same
shifts as the fluid); the D3Q15 ones come from the raw moments by the
aliased binomial shift, and their reverse needs one central moment outside
the set (210).  Above second order the moments relax toward option A, option
B or the Maxwellian (MCM) attractors.  A diagonal thermal link that crosses a
Dirichlet face is anti-bounced toward the mean temperature of the Dirichlet
faces it crosses, so the wall-temperature gradient of an edge or corner link
is shared between two or three faces: the "box" cases (Dirichlet walls on
every face) check that split.

Bars as for the D2Q5 adjoint: one adjoint step and the adjoint of the initial
collision equal the oracle's vector-Jacobian products to 1e-12 (FP64) and
2e-5 (FP32 deviations); a checkpointed gradient equals the oracle's autograd
gradient to 1e-10.  Temperatures are raised by 1.5 so that option B's
division by T stays away from zero.
"""

import ctypes

import pytest
import torch

import workloads
from oracle import gradient as ograd
from oracle import sim as osim
from oracle.params import params_from_config
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

MODELS = [("FP", "A"), ("FP", "B"), ("MCM", "A")]


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _cfg(case):
    if case in ("box2d", "box3d"):
        # Dirichlet walls on every face: corner links cross two (2D) or
        # three (3D) of them
        cfg = G.small_config("dhc2d" if case == "box2d" else "dhc3d")
        temps = [0.2, -0.1, 0.3, -0.25]
        for f in range(2, 4 if case == "box2d" else 6):
            cfg["faces"][f] = {"fluid": "noslip", "thermal": "dirichlet", "T": temps[f - 2], "u_w": (0.0, 0.0, 0.0)}
    else:
        cfg = G.small_config(case)
    return G.with_pair(G.shift_temperature(cfg, 1.5), True)


def _faces(cfg):
    return [f for f, fd in enumerate(cfg["faces"]) if fd["thermal"] == "dirichlet"]


def _profile_shape(cfg, face):
    nx, ny, nz = cfg["shape"]
    return {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[face // 2]


@pytest.mark.parametrize("case", ["dhc2d", "rb2d", "mixed2d", "rb2d_tiles", "box2d",
                                  "dhc3d", "rb3d", "lid3d", "dhc3d_tiles", "box3d"])
@pytest.mark.parametrize("model,opt", MODELS)
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32dev", 2e-5), ("f32uni", 2e-5)])
def test_adjoint_step_matches_oracle_vjp(case, model, opt, precision, tol):
    from paper_2504_09041_amd import _abi as A

    print(f"case={case} model={model} option={opt} precision={precision}", flush=True)
    cfg = _cfg(case)
    kw = dict(model=model, thermal_option=opt)
    prm = params_from_config(cfg, **kw)
    f0, g0 = G.perturbed_state(cfg, seed=71, **kw)
    faces = _faces(cfg)
    face = faces[0] if faces else None
    theta = None
    if face is not None:
        theta = cfg["faces"][face]["T"] + 0.1 * torch.tensor(workloads.uniform_field(_profile_shape(cfg, face), 72))
    Q = f0.shape[0] + g0.shape[0]
    mu = torch.tensor(workloads.uniform_field((Q,) + tuple(f0.shape[1:]), 73))
    dJdT = torch.tensor(workloads.uniform_field(tuple(f0.shape[1:]), 74))
    ke = 0.7
    ref, dth_ref = G.adjoint_step_reference(prm, f0, g0, mu, dJdT, ke, face, theta)
    sim = G.make_sim(cfg, precision, wall_profiles={face: theta} if theta is not None else None, **kw)
    G.load_state(sim, f0, g0)
    S_prev = sim.save()
    dt = torch.float64 if precision == "f64" else torch.float32
    lin = sim.to_storage(mu, dt)
    lout = torch.full_like(lin, float("nan"))
    dth = torch.zeros(theta.shape, dtype=torch.float64, device="cuda") if theta is not None else None
    arr = (ctypes.c_void_p * 6)()
    if dth is not None:
        arr[face] = dth.data_ptr()
    w = dJdT.cuda().contiguous()
    A.check(A.load().fpc_adjoint_step(sim.handle, _ptr(S_prev), _ptr(lin), _ptr(lout), _ptr(w),
                                      ctypes.c_double(ke), arr), "fpc_adjoint_step")
    torch.cuda.synchronize()
    got = sim.from_storage(lout).double().cpu()
    assert torch.isfinite(got).all(), "a slot of mu_{n-1} was not written"
    err = G.rel_err(got, ref)
    print(f"  rel err mu {err:.2e}")
    assert err < tol
    if theta is not None:
        e2 = G.rel_err(dth.cpu(), dth_ref)
        print(f"  rel err dtheta {e2:.2e}")
        assert e2 < tol
    sim.close()


@pytest.mark.parametrize("case", ["dhc2d", "mixed2d", "box2d", "rb3d", "box3d"])
@pytest.mark.parametrize("model,opt", MODELS)
def test_adjoint_init_matches_oracle(case, model, opt):
    from paper_2504_09041_amd import _abi as A

    cfg = _cfg(case)
    kw = dict(model=model, thermal_option=opt)
    prm = params_from_config(cfg, **kw)
    T0 = G.initial_T(cfg) + 0.2 * torch.tensor(workloads.uniform_field(tuple(cfg["shape"][::-1]), 75))
    T = T0.clone().requires_grad_(True)
    fo, go = osim.init_state(prm, T)
    Q = fo.shape[0] + go.shape[0]
    mu = torch.tensor(workloads.uniform_field((Q,) + tuple(fo.shape[1:]), 76))
    lam_f, lam_g = G.pull_transpose(prm, mu[: fo.shape[0]], mu[fo.shape[0]:])
    dJdT = torch.tensor(workloads.uniform_field(tuple(fo.shape[1:]), 77))
    mac = osim.macros_of_state(prm, fo, go)
    L = (lam_f * fo).sum() + (lam_g * go).sum() + (dJdT * mac["T"]).sum() + 0.3 * osim.kinetic_energy(mac)
    (gT,) = torch.autograd.grad(L, [T])
    sim = G.make_sim(cfg, "f64", **kw)
    lin = sim.to_storage(mu, torch.float64)
    out = torch.empty(tuple(fo.shape[1:]), dtype=torch.float64, device="cuda")
    Tc = T0.cuda().contiguous()  # kept alive over the call: the ABI takes raw pointers
    w = dJdT.cuda().contiguous()
    A.check(A.load().fpc_adjoint_init(sim.handle, _ptr(Tc), _ptr(lin), _ptr(w), ctypes.c_double(0.3), _ptr(out)),
            "fpc_adjoint_init")
    torch.cuda.synchronize()
    err = G.rel_err(out.cpu(), gT)
    print(f"case={case} model={model} option={opt}: rel err {err:.2e}")
    assert err < 1e-12
    sim.close()


@pytest.mark.parametrize("case,kind,face,window,tf", [
    # wall Nusselt number of the top lid over levels 10..25, gradient on the
    # bottom-wall profile (whose corner links share the side walls' faces in
    # the box)
    ("mixed2d", "nu", 3, (10, 25), 2),
    ("box2d", "nu", 1, (10, 25), 0),
    ("dhc2d", "ke", None, 20, 0),
    ("box3d", "nu", 1, (10, 25), 0),
    ("rb3d", "ke", None, 20, 4),
])
@pytest.mark.parametrize("model,opt", MODELS)
def test_checkpointed_gradient_matches_oracle_autograd(case, kind, face, window, tf, model, opt):
    from paper_2504_09041_amd import adjoint as adj
    from paper_2504_09041_amd.sim import params_from_workload

    print(f"case={case} kind={kind} model={model} option={opt}", flush=True)
    cfg = _cfg(case)
    kw = dict(model=model, thermal_option=opt)
    prm = params_from_config(cfg, **kw)
    N, K = 25, 6
    shape = cfg["shape"]
    T0 = G.initial_T(cfg) + 0.05 * torch.tensor(workloads.uniform_field(tuple(shape[::-1]), 78))
    th0 = cfg["faces"][tf]["T"] + 0.05 * torch.tensor(workloads.uniform_field(_profile_shape(cfg, tf), 79))
    J_o, gth_o, gT_o = ograd.gradient(prm, T0, N, kind, face=face, window=window if kind == "nu" else None,
                                      theta_face=tf, theta=th0, at=window if kind == "ke" else None)
    p = params_from_workload(cfg, "f64", **kw)
    obj = adj.WallNusselt(face, *window) if kind == "nu" else adj.KineticEnergy(window)
    s = adj.AdjointSolver(p, N, K, obj, theta_face=tf)
    J = s.forward(th0.cuda(), T0.cuda())
    gth, gT = s.backward()
    print(f"  J gpu {J:.15e} oracle {J_o:.15e}")
    assert abs(J - J_o) <= 1e-12 * max(1.0, abs(J_o))
    e1 = G.rel_err(gT.cpu(), gT_o)
    e2 = G.rel_err(gth.cpu(), gth_o)
    print(f"  rel err dJ/dT_init {e1:.2e}  dJ/dtheta {e2:.2e}")
    assert e1 < 1e-10
    assert e2 < 1e-10


@pytest.mark.parametrize("wl,shape,pair,N,K", [
    ("rb3d_128", (32, 32, 32), "D3Q27-D3Q15", 200, 14),
    ("rb2d_1024x512", (128, 64, 1), "D2Q9-D2Q9", 300, 17),
])
def test_gradient_matches_central_differences(wl, shape, pair, N, K):
    """Rayleigh-Benard at 32^3 on the paper's D3Q15 thermal lattice and at
    128 x 64 on its D2Q9 one (FP64, option A): J = kinetic energy at step N,
    gradient with respect to the whole initial temperature field through the
    checkpointed sweep, against central differences of the GPU forward run
    along 4 seeded unit directions (1e-6 relative at the best step h, against
    at least a tenth of the typical |grad| / sqrt(n)) -- sizes the oracle's
    autograd does not reach."""
    from paper_2504_09041_amd import adjoint as adj
    from paper_2504_09041_amd.sim import params_from_workload

    print(f"{wl} {shape} {pair} N={N} K={K}", flush=True)
    cfg = workloads.config(wl, shape=shape, pair=pair)
    T0 = G.initial_T(cfg).cuda()
    s = adj.AdjointSolver(params_from_workload(cfg, "f64"), N, K, adj.KineticEnergy(N))
    J = s.forward(None, T0)
    _, gT = s.backward()
    dirs = torch.tensor(workloads.unit_directions(T0.numel(), 4, seed0=400)).cuda()
    # a random unit direction has a directional derivative of about
    # |grad| / sqrt(n); one far below that is made of cancelling terms, so
    # errors are measured against at least a tenth of it
    floor = 0.1 * float(gT.norm()) / T0.numel() ** 0.5
    worst = 0.0
    for i in range(dirs.shape[0]):
        d = dirs[i].reshape(gT.shape)
        an = float((gT * d).sum())
        best = float("inf")
        for h in (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4):
            fd = (s.forward(None, T0 + h * d) - s.forward(None, T0 - h * d)) / (2 * h)
            best = min(best, abs(fd - an) / max(abs(an), floor))
        print(f"  direction {i}: dJ {an:.6e} (floor {floor:.3e}), best relative error {best:.2e}", flush=True)
        worst = max(worst, best)
    print(f"J {J:.6e}; worst directional relative error {worst:.2e}")
    assert worst < 1e-6
    s.sim.close()
