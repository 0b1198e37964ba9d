"""The wall-Nusselt objective entry points (through the C ABI) against the
diagnostics and the oracle.

* fpc_step_nusselt: steps bit-identical to fpc_step, and its accumulated
  sum of weight * <Nu>_face(n) equals weight times the fpc_diagnostics
  values of the same levels (1e-12 relative: FP64 sums in another order),
  on every kind of face, including an x face whose two wall layers lie in
  different 64-node tiles;
* fpc_nusselt_seed: the adjoint seeds equal the oracle's autograd gradient
  of weight * <Nu>_face (Sec. 6.1 stencil) with respect to T and the wall
  temperature profile;
* fpc_nusselt_local: the local wall Nusselt numbers, whose mean is the
  oracle's <Nu>.
"""

import pytest
import torch

import workloads
from oracle import sim as osim
from oracle.params import params_from_config
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


def _cfg(case):
    if case == "dhc2d_x129":
        # hot -x / cold +x walls, 129 nodes across: the +x wall layers x = 128
        # and x = 127 lie in different storage tiles
        return workloads.config("dhc2d_64", shape=(129, 6, 1))
    return G.small_config(case)


CASES = [("dhc2d_x129", 0), ("dhc2d_x129", 1), ("mixed2d", 2), ("mixed2d", 3), ("rb2d_tiles", 2),
         ("dhc3d_tiles", 1), ("lid3d", 5), ("rb3d", 4)]


@pytest.mark.parametrize("case,face", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32dev"])
def test_step_nusselt_accumulates_the_diagnostics(case, face, precision):
    print(f"case={case} face={face} precision={precision}", flush=True)
    cfg = _cfg(case)
    f0, g0 = G.perturbed_state(cfg, seed=61)
    weight, n = 0.37, 20
    a = G.make_sim(cfg, precision)
    G.load_state(a, f0, g0)
    acc = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    a.step_nusselt(n // 2, face, weight, acc)
    a.step_nusselt(n - n // 2, face, weight, acc)
    b = G.make_sim(cfg, precision)
    G.load_state(b, f0, g0)
    ref = 0.25
    for _ in range(n):
        b.step(1)
        ref += weight * b.diagnostics(face)["nu"]
    got = float(acc.item())
    print(f"  acc {got:.15e} ref {ref:.15e}")
    assert abs(got - ref) <= 1e-12 * abs(ref)
    ib = torch.int64 if precision == "f64" else torch.int32
    assert torch.equal(a.state_populations().view(ib), b.state_populations().view(ib))
    assert a.step_count == b.step_count == n
    a.close()
    b.close()


@pytest.mark.parametrize("case,face", [("mixed2d", 2), ("dhc2d_x129", 1), ("lid3d", 5), ("dhc3d_tiles", 0)])
def test_nusselt_seed_is_the_oracle_gradient(case, face):
    cfg = _cfg(case)
    prm = params_from_config(cfg)
    nx, ny, nz = cfg["shape"]
    k = face // 2
    shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[k]
    T = G.initial_T(cfg) + 0.3 * torch.tensor(workloads.uniform_field((nz, ny, nx), 62))
    Tw = cfg["faces"][face]["T"] + 0.1 * torch.tensor(workloads.uniform_field(shp, 63))
    weight = 0.7
    Tr = T.clone().requires_grad_(True)
    Twr = Tw.clone().requires_grad_(True)
    J = weight * osim.nusselt(prm, Tr, face, {face: Twr})
    gT, gTw = torch.autograd.grad(J, [Tr, Twr])
    sim = G.make_sim(cfg, "f64", wall_profiles={face: Tw})
    dT, dTw = sim.nusselt_seed(face, weight)
    assert G.rel_err(dT.cpu(), gT) < 1e-15
    assert G.rel_err(dTw.cpu().reshape(shp), gTw) < 1e-15
    sim.close()


@pytest.mark.parametrize("case,face", [("dhc2d_x129", 0), ("mixed2d", 3), ("dhc3d_tiles", 1), ("rb3d", 5)])
def test_local_nusselt_numbers(case, face):
    cfg = _cfg(case)
    f0, g0 = G.perturbed_state(cfg, seed=64)
    sim = G.make_sim(cfg, "f64")
    G.load_state(sim, f0, g0)
    sim.step(5)
    loc = sim.nusselt_local(face).cpu()
    fo, go, mac, prm = G.oracle_run(cfg, f0, g0, 5)
    nu_o = float(osim.nusselt(prm, mac["T"], face))
    assert abs(float(loc.mean()) - nu_o) <= 1e-12 * max(1.0, abs(nu_o))
    # the stencil per node, from the oracle's time-level temperature
    k = face // 2
    n = cfg["shape"][k]
    dim = 2 - k
    l0, l1 = (0, 1) if face % 2 == 0 else (n - 1, n - 2)
    T1, T2 = mac["T"].select(dim, l0), mac["T"].select(dim, l1)
    ref = -(n / prm.dT_ref) * (-8.0 / 3.0 * cfg["faces"][face]["T"] + 3.0 * T1 - T2 / 3.0)
    assert G.rel_err(loc, ref.reshape(loc.shape)) < 1e-12
    assert abs(sim.diagnostics(face)["nu"] - float(loc.mean())) <= 1e-13 * max(1.0, abs(nu_o))
    sim.close()
