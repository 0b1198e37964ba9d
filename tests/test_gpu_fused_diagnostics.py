"""fpc_step_diagnostics (through the C ABI) against fpc_step + the diagnostics.

The fused entry point advances n steps and lets the kernel of the last step
reduce the diagnostics of the state it writes over each 64-node tile; two
small kernels reduce the tiles.  Its reference is the same n steps taken as
fpc_step(n - 1) then fpc_step(1) (the launches the fused call makes), followed
by the separate diagnostics pass over the stored state:

* the states are bit-identical (the fused step is the same kernel; the
  diagnostics run after its stores);
* KE, sum T, max |u| and the wall Nusselt number agree to the order of the
  FP64 sums (1e-13 relative, sum T against the sum of |T|), the count of
  non-finite nodes exactly;
* in FP64 storage, they equal the oracle's diagnostics of the same level;
* on 2D and 3D, FP64 and FP32 storage, the paper's thermal lattices, rows of
  several tiles with a ragged last tile, grids past the multi-step path's
  size, several steps per call, and a state holding a NaN.
"""

import ctypes

import pytest
import torch

import workloads
from oracle import sim as osim
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


def _noalloc(sim, face):
    from paper_2504_09041_amd import _abi as A

    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    A.check(A.load().fpc_diagnostics_noalloc(sim.handle, face, ctypes.c_void_p(out.data_ptr())),
            "fpc_diagnostics_noalloc")
    torch.cuda.synchronize()
    return out.cpu().tolist()


def _sum_abs_T(sim):
    return float(sim.macros()["T"].abs().sum())


def _compare(got, ref, sumabsT):
    print(f"  fused {got}\n  ref   {ref}", flush=True)
    nu, ke, st, um, bad = got
    assert abs(nu - ref[0]) <= 1e-12 * max(abs(ref[0]), 1.0)
    assert abs(ke - ref[1]) <= 1e-13 * abs(ref[1])
    assert abs(st - ref[2]) <= 1e-13 * sumabsT
    assert abs(um - ref[3]) <= 1e-13 * abs(ref[3])
    assert bad == ref[4]


def _pair(a, b, precision):
    ib = torch.int64 if precision == "f64" else torch.int32
    assert torch.equal(a.state_populations().view(ib), b.state_populations().view(ib))
    assert a.step_count == b.step_count
    assert a.multistep_launches == b.multistep_launches


CASES = [
    # (small case, paper thermal lattice, steps)
    ("dhc2d", False, 1),
    ("mixed2d", False, 7),
    ("rb2d_tiles", False, 5),
    ("dhc3d", False, 3),
    ("dhc3d_tiles", False, 4),
    ("lid3d", False, 2),
    ("rb3d", False, 6),
    ("dhc2d", True, 3),
    ("dhc3d", True, 2),
]


@pytest.mark.parametrize("case,paper_thermal,n", CASES)
@pytest.mark.parametrize("precision", ["f64", "f32dev"])
def test_fused_diagnostics_equal_the_separate_pass(case, paper_thermal, n, precision):
    print(f"case={case} paper_thermal={paper_thermal} n={n} precision={precision}", flush=True)
    cfg = G.with_pair(G.small_config(case), paper_thermal)
    f0, g0 = G.perturbed_state(cfg, seed=83)
    for face in (cfg["nu_face"], -1):
        a = G.make_sim(cfg, precision)
        G.load_state(a, f0, g0)
        got = a.step_diagnostics(n, face).cpu().tolist()
        b = G.make_sim(cfg, precision)
        G.load_state(b, f0, g0)
        if n > 1:
            b.step(n - 1)
        b.step(1)
        ref = _noalloc(b, face)
        _pair(a, b, precision)
        assert a.step_count == n
        _compare(got, ref, _sum_abs_T(b))
        if face < 0:
            assert got[0] == 0.0
        assert got[1] > 0.0 and got[3] > 0.0 and got[4] == 0.0
        if precision == "f64":
            # and the oracle's diagnostics of the same time level
            _, _, mac, prm = G.oracle_run(cfg, f0, g0, n)
            tol = 1e-12
            if face >= 0:
                nu_o = float(osim.nusselt(prm, mac["T"], face))
                assert abs(got[0] - nu_o) <= tol * max(1.0, abs(nu_o))
            ke_o = float(osim.kinetic_energy(mac))
            assert abs(got[1] - ke_o) <= 1e-9 * ke_o
            assert abs(got[2] - float(mac["T"].sum())) <= tol * float(mac["T"].abs().sum())
            um_o = float(mac["u"].pow(2).sum(0).sqrt().max())
            assert abs(got[3] - um_o) <= 10 * tol
        a.close()
        b.close()


@pytest.mark.parametrize("wl,shape,precision,n", [
    # several hundred tiles (3D FP32, non-temporal stores off) and a 2D grid
    # with ragged rows, both beyond the single-launch multi-step path
    ("dhc3d_256", (128, 64, 48), "f32dev", 4),
    ("rb2d_1024x512", (300, 100, 1), "f64", 3),
])
def test_fused_diagnostics_on_larger_grids(wl, shape, precision, n):
    print(f"{wl} {shape} {precision} n={n}", flush=True)
    cfg = workloads.config(wl, shape=shape)
    T = G.initial_T(cfg) + 0.05 * torch.tensor(workloads.uniform_field(tuple(shape[::-1]), 5))
    a = G.make_sim(cfg, precision)
    b = G.make_sim(cfg, precision)
    a.init(T.cuda())
    b.init(T.cuda())
    a.step(10)
    b.step(10)
    face = cfg["nu_face"]
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    # two calls into the same output: the second overwrites the first
    a.step_diagnostics(n, face, out)
    got = a.step_diagnostics(n, face, out).cpu().tolist()
    b.step(2 * n)
    ref = _noalloc(b, face)
    _pair(a, b, precision)
    _compare(got, ref, _sum_abs_T(b))
    assert got[1] > 0.0 and got[4] == 0.0
    a.close()
    b.close()


@pytest.mark.parametrize("case,face", [("mixed2d", 3), ("rb2d_tiles", 2), ("dhc3d_tiles", 1)])
@pytest.mark.parametrize("precision", ["f64", "f32dev"])
def test_fused_diagnostics_with_a_wall_temperature_profile(case, face, precision):
    """A per-node Dirichlet temperature on the Nusselt face: the fused wall
    term reads the profile as the separate pass does."""
    print(f"case={case} face={face} precision={precision}", flush=True)
    cfg = G.small_config(case)
    nx, ny, nz = cfg["shape"]
    shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[face // 2]
    Tw = cfg["faces"][face]["T"] + 0.1 * torch.tensor(workloads.uniform_field(shp, 91))
    f0, g0 = G.perturbed_state(cfg, seed=92)
    a = G.make_sim(cfg, precision, wall_profiles={face: Tw})
    b = G.make_sim(cfg, precision, wall_profiles={face: Tw})
    G.load_state(a, f0, g0)
    G.load_state(b, f0, g0)
    got = a.step_diagnostics(3, face).cpu().tolist()
    b.step(2)
    b.step(1)
    ref = _noalloc(b, face)
    _pair(a, b, precision)
    _compare(got, ref, _sum_abs_T(b))
    a.close()
    b.close()


@pytest.mark.parametrize("case", ["rb2d_tiles", "dhc3d_tiles"])
@pytest.mark.parametrize("precision", ["f64", "f32dev"])
def test_fused_diagnostics_count_non_finite_nodes(case, precision):
    cfg = G.small_config(case)
    f0, g0 = G.perturbed_state(cfg, seed=89)
    nx, ny, nz = cfg["shape"]
    # one NaN population at an interior node of the second tile: after one
    # step the node and the neighbours that pull from it hold NaN macros
    f0 = f0.clone()
    f0[1, nz // 2, ny // 2, 70] = float("nan")
    print(f"case={case} precision={precision}: NaN at x=70", flush=True)
    a = G.make_sim(cfg, precision)
    G.load_state(a, f0, g0)
    got = a.step_diagnostics(1, cfg["nu_face"]).cpu().tolist()
    b = G.make_sim(cfg, precision)
    G.load_state(b, f0, g0)
    b.step(1)
    ref = _noalloc(b, cfg["nu_face"])
    assert ref[4] >= 1.0
    assert got[4] == ref[4]
    assert abs(got[1] - ref[1]) <= 1e-13 * abs(ref[1])
    assert abs(got[3] - ref[3]) <= 1e-13 * abs(ref[3])
    a.close()
    b.close()


def test_fused_diagnostics_rejects_bad_arguments():
    from paper_2504_09041_amd import _abi as A

    cfg = G.small_config("rb2d")  # periodic x faces
    sim = G.make_sim(cfg, "f64")
    sim.init(G.initial_T(cfg).cuda())
    lib = A.load()
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(out.data_ptr())
    assert lib.fpc_step_diagnostics(sim.handle, 0, -1, p) == A.FPC_ERR_ARG
    assert lib.fpc_step_diagnostics(sim.handle, 1, 2, None) == A.FPC_ERR_ARG
    assert lib.fpc_step_diagnostics(sim.handle, 1, 6, p) == A.FPC_ERR_ARG
    assert lib.fpc_step_diagnostics(sim.handle, 1, 0, p) == A.FPC_ERR_STATE  # periodic x face
    assert lib.fpc_step_diagnostics(sim.handle, 1, 4, p) == A.FPC_ERR_STATE  # 2D has no z faces
    assert sim.step_count == 0  # nothing advanced
    sim.close()
