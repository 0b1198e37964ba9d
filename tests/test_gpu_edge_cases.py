"""Edge cases of the HIP path against the FP64 oracle: degenerate grid widths
(one node across a periodic axis, the minimum of two nodes between two walls
or between a wall and a moving lid), rows that fill exactly one storage tile or spill one node into a
second, zero steps, and states above 4 GiB (the 64-bit addressing path of the
step kernels).

Bars as in the parity tests: FP64 within 1e-13 after one step and 1e-12 after
100 steps; FP32 deviations within the sampled full-size bar.
"""

import pytest
import torch

import workloads
from oracle import sim as osim
from oracle.collision import rest_weights
from oracle.params import params_from_config
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


# (workload, shape): which axes are periodic / walled follows the workload
DEGENERATE = {
    "rb2d_nx1": ("rb2d_1024x512", (1, 6, 1)),        # one node across the periodic x axis
    "dhc2d_nx2": ("dhc2d_64", (2, 5, 1)),            # two nodes between the two x walls
    "mixed2d_ny2": ("mixed2d_512", (5, 2, 1)),       # two rows between the bottom wall and the lid
    "rb3d_1x1": ("rb3d_128", (1, 1, 5)),             # one column, periodic x and y of width 1
    "rb3d_nz2": ("rb3d_128", (3, 2, 2)),             # two layers between the z walls
    "dhc3d_2x2x2": ("dhc3d_256", (2, 2, 2)),         # walls on every face, two nodes per axis
    "rb2d_nx64": ("rb2d_1024x512", (64, 3, 1)),      # one full tile per row, periodic x
    "dhc2d_nx65": ("dhc2d_64", (65, 3, 1)),          # a second tile holding one node, x walls
    "rb3d_nx65": ("rb3d_128", (65, 3, 3)),           # the same in 3D, periodic x
}


@pytest.mark.parametrize("case", list(DEGENERATE))
@pytest.mark.parametrize("nsteps,tol", [(1, 1e-13), (100, 1e-12)])
def test_degenerate_grids_match_oracle(case, nsteps, tol):
    print(f"case={case} nsteps={nsteps}", flush=True)
    wl, shape = DEGENERATE[case]
    cfg = workloads.config(wl, shape=shape)
    f0, g0 = G.perturbed_state(cfg, seed=41)
    sim = G.make_sim(cfg, "f64")
    G.load_state(sim, f0, g0)
    sim.step(nsteps)
    f, g = G.read_state(sim)
    fo, go, mac, prm = G.oracle_run(cfg, f0, g0, nsteps)
    assert G.rel_err(f, fo) < tol
    assert G.rel_err(g, go) < tol
    m = sim.macros()
    assert G.rel_err(m["T"].cpu(), mac["T"]) < tol
    sim.close()


@pytest.mark.parametrize("case", ["rb2d_nx1", "dhc3d_2x2x2", "dhc2d_nx65"])
def test_degenerate_grids_fp32_deviation(case):
    """FP32 deviation storage on the degenerate grids, 100 steps, with the
    bars of the small parity cases (populations 1e-5 of their scale, T within
    1e-4 of the temperature difference)."""
    wl, shape = DEGENERATE[case]
    cfg = workloads.config(wl, shape=shape)
    f0, g0 = G.perturbed_state(cfg, seed=43)
    sim = G.make_sim(cfg, "f32dev")
    G.load_state(sim, f0, g0)
    sim.step(100)
    f, g = G.read_state(sim)
    fo, go, mac, _ = G.oracle_run(cfg, f0, g0, 100)
    assert G.rel_err(f, fo) < 1e-5
    assert G.rel_err(g, go) < 1e-5
    dT = cfg["T_hot"] - cfg["T_cold"]
    assert float((sim.macros()["T"].cpu() - mac["T"]).abs().max()) < 1e-4 * dT
    sim.close()


def test_zero_steps_leave_the_state_alone():
    cfg = workloads.config("dhc2d_64", shape=(70, 5, 1))
    f0, g0 = G.perturbed_state(cfg, seed=45)
    sim = G.make_sim(cfg, "f64")
    G.load_state(sim, f0, g0, step=3)
    before = sim.save()
    sim.step(0)
    torch.cuda.synchronize()
    assert sim.step_count == 3
    assert torch.equal(sim.save(), before)
    sim.close()


@pytest.mark.parametrize("workload,precision,shape,tol", [
    ("dhc3d_256", "f32dev", (320, 320, 320), 2e-6),    # 4.46 GB per state buffer
    ("rb2d_1024x512", "f64", (6400, 6400, 1), 1e-13),  # 4.59 GB per state buffer
])
def test_state_above_4GiB_on_sampled_nodes(workload, precision, shape, tol):
    """One step of a state larger than 4 GiB (64-bit element offsets instead
    of buffer descriptors), checked at ~2000 sampled nodes plus corners and
    face bands; then one step with fused diagnostics against the separate
    pass."""
    print(f"workload={workload} precision={precision} shape={shape}", flush=True)
    cfg = workloads.config(workload, shape=shape)
    prm = params_from_config(cfg)
    lf, lg = prm.lattices
    wf = rest_weights(lf)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    sim = G.make_sim(cfg, precision)
    assert sim.nbytes >= 4 * 1024 ** 3
    S = G.full_hashed_state(shape, lf.Q, lg.Q, wf, wg, seed=47, device="cuda")
    sim.import_fp64(S)
    del S
    sim.step(1)
    out = sim.export_fp64()
    x, y, z = G.sample_nodes(shape, 2000, seed=48)
    got = out[:, z.cuda(), y.cuda(), x.cuda()].cpu()
    del out
    gf, gg = G.hashed_state_getters(shape, lf.Q, lg.Q, wf, wg, seed=47)
    fo, go, _ = osim.step_at(prm, gf, gg, (x, y, z))
    assert G.rel_err(got[: lf.Q], fo) < tol
    assert G.rel_err(got[lf.Q:], go) < tol
    # the diagnostics fused into a step on the 64-bit addressing path equal
    # the separate pass over the state that step writes
    import ctypes

    from paper_2504_09041_amd import _abi as A

    face = cfg["nu_face"]
    fused = sim.step_diagnostics(1, face).cpu().tolist()
    ref = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    A.check(A.load().fpc_diagnostics_noalloc(sim.handle, face, ctypes.c_void_p(ref.data_ptr())),
            "fpc_diagnostics_noalloc")
    ref = ref.cpu().tolist()
    sum_abs_T = float(sim.macros()["T"].abs().sum())
    print(f"  fused {fused}\n  ref   {ref}")
    assert abs(fused[0] - ref[0]) <= 1e-12 * max(1.0, abs(ref[0]))
    assert abs(fused[1] - ref[1]) <= 1e-13 * abs(ref[1])
    assert abs(fused[2] - ref[2]) <= 1e-13 * sum_abs_T
    assert abs(fused[3] - ref[3]) <= 1e-13 * abs(ref[3])
    assert fused[4] == ref[4]
    sim.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("wl,n", [("dhc3d_256", 8), ("rb3d_128", 8), ("dhc3d_256", 16), ("rb3d_128", 16)])
def test_cubes_match_oracle(wl, n):
    """8^3 and 16^3 boxes (walls on every face, or periodic x / y), 100 FP64
    steps: every node against the oracle."""
    print(f"workload={wl} n={n}", flush=True)
    cfg = workloads.config(wl, shape=(n, n, n))
    f0, g0 = G.perturbed_state(cfg, seed=49)
    sim = G.make_sim(cfg, "f64")
    G.load_state(sim, f0, g0)
    sim.step(100)
    f, g = G.read_state(sim)
    fo, go, _, _ = G.oracle_run(cfg, f0, g0, 100)
    assert G.rel_err(f, fo) < 1e-12
    assert G.rel_err(g, go) < 1e-12
    sim.close()


def test_fp32_default_meets_the_bars_over_the_full_run():
    """2D Rayleigh-Benard 1024x512, Ra 1e6, from the same initial field over
    the workload's full 50,000 steps: the FP32 deviation form with the
    library's default storage reference against the GPU FP64 run (itself
    pinned to the oracle), checked every 5,000 steps against the bars of
    1e-4 of the temperature difference on T and 1e-3 relative on the
    bottom-wall Nusselt number."""
    cfg = workloads.config("rb2d_1024x512")
    T0 = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    sims = {}
    for prec in ("f64", "f32dev"):
        sims[prec] = G.make_sim(cfg, prec)
        sims[prec].init(T0)
    dT = cfg["T_hot"] - cfg["T_cold"]
    worst_T = worst_Nu = 0.0
    for n in range(5000, 50001, 5000):
        out = {}
        for prec, sim in sims.items():
            sim.step(5000)
            out[prec] = (sim.macros()["T"], sim.diagnostics(cfg["nu_face"])["nu"])
        eT = float((out["f32dev"][0] - out["f64"][0]).abs().max()) / dT
        eNu = abs(out["f32dev"][1] - out["f64"][1]) / abs(out["f64"][1])
        worst_T, worst_Nu = max(worst_T, eT), max(worst_Nu, eNu)
        print(f"step {n}: max|dT|/DeltaT {eT:.2e}, rel dNu {eNu:.2e}", flush=True)
        assert eT < 1e-4
        assert eNu < 1e-3
    for sim in sims.values():
        sim.close()
    print(f"worst over the run: {worst_T:.2e} / {worst_Nu:.2e}")
