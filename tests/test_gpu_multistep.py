"""fpc_step's single-launch multi-step path on small grids.

Small grids (at most 16 blocks of 256 nodes, any lattice pair in 2D or in 3D
FP32, the standard rate set) advance up to 1024 steps per
cooperative launch with a grid-wide barrier between the steps.  Each step is
the arithmetic of the one-launch-per-step kernel; the two kernels are
compiled separately, so the compiler may fuse multiply-adds differently and
the states agree to rounding, not bit for bit.  The bars below are the
oracle bars (FP64 1e-12 relative; FP32 populations 1e-5 of their scale, T
1e-4 dT, Nu 1e-3): both paths must meet them against the oracle, which the
100-step parity tests and the 2000-step 64^2 cavity run of
test_gpu_parity.py check for this path directly (they run through it).
"""

import pytest
import torch

from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


# (small case or workload name, shape, precision)
CASES = [
    ("dhc2d_64", (64, 64, 1), "f64"),     # the 64^2 cavity itself
    ("rb2d_tiles", None, "f64"),          # periodic x, ragged last tile
    ("rb2d_tiles", None, "f32dev"),
    ("mixed2d", None, "f32dev"),          # moving lid, Dirichlet profile walls
    ("rb2d_1024x512", (256, 16, 1), "f32dev"),  # 16 working blocks, the largest grid of the path
    ("dhc3d", None, "f32dev"),
    ("dhc3d_tiles", None, "f32uni"),
    ("rb3d_128", (8, 8, 8), "f32dev"),  # periodic x and y
    ("lid3d", None, "f32dev"),
    # the paper's thermal lattices (D2Q9 in 2D, D3Q15 in 3D)
    ("dhc2d_64:paper", (64, 64, 1), "f64"),
    ("mixed2d:paper", None, "f32dev"),
    ("dhc3d:paper", None, "f32dev"),
    ("rb3d_128:paper", (8, 8, 8), "f32dev"),
]


def _config(name, shape):
    import workloads

    base, _, paper = name.partition(":")
    cfg = G.small_config(base) if shape is None else workloads.config(base, shape=shape)
    return G.with_pair(cfg, paper == "paper")


def _run(cfg, precision, nsteps, multistep):
    f0, g0 = G.perturbed_state(cfg, seed=5)
    sim = G.make_sim(cfg, precision)
    sim.set_multistep(multistep)
    G.load_state(sim, f0, g0)
    for n in nsteps:
        sim.step(n)
    f, g = G.read_state(sim)
    T = sim.macros()["T"].cpu()
    launches = sim.multistep_launches
    d = sim.diagnostics(cfg["nu_face"])
    sim.close()
    return f, g, T, launches, d


@pytest.mark.parametrize("name,shape,precision", CASES)
def test_multistep_matches_per_step_launches(name, shape, precision):
    cfg = _config(name, shape)
    print(f"case={name} shape={shape} precision={precision}", flush=True)
    # odd and even counts and one step alone (an ordinary launch); in FP64 a
    # count above one launch's 1024 steps (1024 + 76), in FP32 a shorter run
    # (its rounding differences are barely damped on the smallest grids)
    long = 1100 if precision == "f64" else 150
    nsteps = (1, 2, 7, 40, long)
    fa, ga, Ta, la, da = _run(cfg, precision, nsteps, True)
    fb, gb, Tb, lb, db = _run(cfg, precision, nsteps, False)
    assert lb == 0
    assert la == (5 if long > 1024 else 4)
    if precision == "f64":
        assert G.rel_err(fa, fb) < 1e-12
        assert G.rel_err(ga, gb) < 1e-12
        assert abs(da["nu"] - db["nu"]) <= 1e-12 * abs(db["nu"])
    else:
        assert G.rel_err(fa, fb) < 1e-5
        assert G.rel_err(ga, gb) < 1e-5
        assert float((Ta - Tb).abs().max()) < 1e-4 * (cfg["T_hot"] - cfg["T_cold"])
        assert abs(da["nu"] - db["nu"]) <= 1e-3 * max(abs(db["nu"]), 1e-3)
    assert not da["unstable"] and not db["unstable"]


@pytest.mark.parametrize("wl,shape,precision", [
    ("dhc2d_64", (64, 68, 1), "f64"),       # 17 working blocks
    ("dhc2d_64", (128, 128, 1), "f32dev"),  # 64
    ("rb3d_128", (16, 16, 16), "f32dev"),   # 64
    ("dhc3d_256", (6, 5, 4), "f64"),        # 3D FP64
])
def test_multistep_path_skips_larger_grids_and_3d_fp64(wl, shape, precision):
    import workloads

    cfg = workloads.config(wl, shape=shape)
    sim = G.make_sim(cfg, precision)
    sim.init(G.initial_T(cfg).cuda())
    sim.step(3)
    assert sim.multistep_launches == 0
    sim.close()


def test_multistep_path_skips_general_rates():
    import workloads

    cfg = workloads.config("dhc2d_64")
    p = G.workload_params(cfg, "f64")
    p.omega_f[6] = 1.1  # a third-order slot off the standard set
    from paper_2504_09041_amd.sim import Simulation

    sim = Simulation(p)
    sim.init(G.initial_T(cfg).cuda())
    sim.step(3)
    assert sim.multistep_launches == 0
    sim.close()


def test_multistep_wait_limit_reports_the_failure_and_falls_back():
    """Failure path of the multi-step launch, forced from the host: with a
    wait limit of 0 a barrier wait gives up at its first unmet check (over
    1000 steps some block always finishes a step before a neighbour), raises
    the error flag, and every block leaves its launch normally.  The next
    diagnostics call reports FPC_ERR_HIP; the sim then runs one launch per
    step, bit-identical to a sim that never used the path."""
    import ctypes

    import workloads
    from paper_2504_09041_amd import _abi as A

    lib = A.load()
    cfg = workloads.config("dhc2d_64")
    T = G.initial_T(cfg).cuda()
    sim = G.make_sim(cfg, "f64")
    sim.init(T)
    A.check(lib.fpc_set_multistep_wait_limit(sim.handle, 0), "fpc_set_multistep_wait_limit")
    sim.step(1000)
    d = [ctypes.c_double() for _ in range(4)]
    rc = lib.fpc_diagnostics(sim.handle, 0, *[ctypes.byref(v) for v in d])
    assert rc == A.FPC_ERR_HIP
    assert "barrier" in A.last_error()
    # the path is off now: a fresh start runs one launch per step
    n0 = sim.multistep_launches
    sim.init(T)
    sim.step(100)
    assert sim.multistep_launches == n0
    assert not sim.diagnostics(0)["unstable"]
    ref = G.make_sim(cfg, "f64")
    ref.set_multistep(False)
    ref.init(T)
    ref.step(100)
    assert torch.equal(sim.export_fp64(), ref.export_fp64())
    sim.close()
    ref.close()

