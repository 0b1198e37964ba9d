"""Parity of the HIP path with the FP64 oracle beyond the hot path's lattices.

The rows checked here:
- the paper's own thermal lattices, D2Q9 (Sec. 4.4, App. B) and D3Q15
  (Sec. 5.4, App. C), with option A and option B for the thermal attractors
  above second order (Eq. Dij2D_goptionA, Eq. Dij2D_g);
- the Maxwellian central-moment comparator (MCM, Sec. 7), on the paper's
  thermal lattices and on the hot path's D2Q5 / D3Q7 pairs.

Bars as for the hot path: FP64 within 1e-13 relative after one step and
1e-12 after 50 steps; FP32 deviations (on every lattice pair) within 1e-5 on
the populations.
Temperatures are raised by 1.5 so that option B's division by T stays away
from zero (the paper's cavity runs use walls at 1 and 2).
"""

import pytest
import torch

import workloads
from oracle import sim as osim
from oracle.collision import rest_weights
from oracle.params import params_from_config
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

CASES = list(G.SMALL_CASES)


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


def _run_and_compare(cfg, precision, kw, seed, tol1, tol50):
    f0, g0 = G.perturbed_state(cfg, seed=seed, **kw)
    sim = G.make_sim(cfg, precision, **kw)
    G.load_state(sim, f0, g0)
    sim.step(1)
    f, g = G.read_state(sim)
    fo, go, mac, prm = G.oracle_run(cfg, f0, g0, 1, **kw)
    e1 = (G.rel_err(f, fo), G.rel_err(g, go))
    sim.step(49)
    f, g = G.read_state(sim)
    fo, go, mac, prm = G.oracle_run(cfg, fo, go, 49, **kw)
    e50 = (G.rel_err(f, fo), G.rel_err(g, go))
    print(f"  1 step {e1[0]:.2e} {e1[1]:.2e}; 50 steps {e50[0]:.2e} {e50[1]:.2e}")
    assert max(e1) < tol1
    assert max(e50) < tol50
    # diagnostics of the time level
    m = sim.macros()
    assert G.rel_err(m["T"].cpu(), mac["T"]) < tol50
    d = sim.diagnostics(cfg["nu_face"])
    nu_o = float(osim.nusselt(prm, mac["T"], cfg["nu_face"]))
    tol_nu = tol50 if precision == "f64" else 1e-3
    assert abs(d["nu"] - nu_o) <= tol_nu * max(1.0, abs(nu_o))
    sim.close()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("model,opt", [("FP", "A"), ("FP", "B"), ("MCM", "A")])
def test_paper_thermal_lattice_steps_match_oracle(case, model, opt):
    print(f"case={case} model={model} option={opt}", flush=True)
    cfg = G.with_pair(G.shift_temperature(G.small_config(case), 1.5), True)
    _run_and_compare(cfg, "f64", dict(model=model, thermal_option=opt), 51, 1e-13, 1e-12)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision,tol1,tol50", [("f64", 1e-13, 1e-12), ("f32cond", 1e-5, 1e-5)])
def test_mcm_on_hot_path_lattices_matches_oracle(case, precision, tol1, tol50):
    print(f"case={case} precision={precision}", flush=True)
    cfg = G.small_config(case)
    _run_and_compare(cfg, precision, dict(model="MCM", thermal_option="A"), 52, tol1, tol50)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("model,opt", [("FP", "A"), ("FP", "B"), ("MCM", "A")])
@pytest.mark.parametrize("precision", ["f32dev", "f32uni"])
def test_paper_thermal_lattice_fp32_matches_oracle(case, model, opt, precision):
    """The FP32 deviation form on the paper's thermal lattices (g stored as
    g - w^T Tr, collided as deviations from the weights' central moments),
    with the default (conduction) and the uniform storage reference."""
    print(f"case={case} model={model} option={opt} precision={precision}", flush=True)
    cfg = G.with_pair(G.shift_temperature(G.small_config(case), 1.5), True)
    _run_and_compare(cfg, precision, dict(model=model, thermal_option=opt), 53, 1e-5, 1e-5)


@pytest.mark.parametrize("workload,pair,precision", [
    ("rb2d_1024x512", "D2Q9-D2Q9", "f32dev"),
    ("rb2d_1024x512", "D2Q9-D2Q9", "f32uni"),
    ("rb3d_128", "D3Q27-D3Q15", "f32dev"),
])
def test_paper_thermal_fp32_full_size_step_on_sampled_nodes(workload, pair, precision):
    """One FP32-deviation step at the full workload size against the oracle
    at ~2000 sampled nodes, at the FP32 bar of the hot path's lattices."""
    print(f"workload={workload} pair={pair} precision={precision}", flush=True)
    cfg = workloads.config(workload, pair=pair)
    prm = params_from_config(cfg)
    lf, lg = prm.lattices
    wf = rest_weights(lf)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    sim = G.make_sim(cfg, precision)
    S = G.full_hashed_state(cfg["shape"], lf.Q, lg.Q, wf, wg, seed=25, device="cuda")
    sim.import_fp64(S)
    del S
    sim.step(1)
    out = sim.export_fp64()
    x, y, z = G.sample_nodes(cfg["shape"], 2000, seed=26)
    got = out[:, z.cuda(), y.cuda(), x.cuda()].cpu()
    del out
    gf, gg = G.hashed_state_getters(cfg["shape"], lf.Q, lg.Q, wf, wg, seed=25)
    fo, go, _ = osim.step_at(prm, gf, gg, (x, y, z))
    ef, eg = G.rel_err(got[: lf.Q], fo), G.rel_err(got[lf.Q:], go)
    print(f"  rel err f {ef:.2e} g {eg:.2e}")
    assert ef < 2e-6
    assert eg < 2e-6
    sim.close()


def test_paper_thermal_fp32_meets_the_bars_over_a_long_run():
    """2D Rayleigh-Benard on the paper's D2Q9 thermal lattice, 256x128,
    Ra 1e5, 20,000 steps from the same initial field: the FP32 deviation form
    (default storage reference) against the GPU FP64 run, every 5,000 steps,
    at the bars of 1e-4 of the temperature difference on T and 1e-3 relative
    on the bottom-wall Nusselt number."""
    cfg = workloads.config("rb2d_1024x512", shape=(256, 128, 1), pair="D2Q9-D2Q9", Ra=1e5)
    T0 = torch.tensor(workloads.initial_temperature(cfg), device="cuda")
    sims = {}
    for prec in ("f64", "f32dev"):
        sims[prec] = G.make_sim(cfg, prec)
        sims[prec].init(T0)
    dT = cfg["T_hot"] - cfg["T_cold"]
    for n in range(5000, 20001, 5000):
        out = {}
        for prec, sim in sims.items():
            sim.step(5000)
            out[prec] = (sim.macros()["T"], sim.diagnostics(cfg["nu_face"])["nu"])
        eT = float((out["f32dev"][0] - out["f64"][0]).abs().max()) / dT
        eNu = abs(out["f32dev"][1] - out["f64"][1]) / abs(out["f64"][1])
        print(f"step {n}: Nu {out['f64'][1]:.6f}, max|dT|/DeltaT {eT:.2e}, rel dNu {eNu:.2e}", flush=True)
        assert eT < 1e-4
        assert eNu < 1e-3
    for sim in sims.values():
        sim.close()


@pytest.mark.parametrize("workload,pair", [("rb2d_1024x512", "D2Q9-D2Q9"), ("dhc3d_256", "D3Q27-D3Q15")])
def test_paper_thermal_full_size_step_on_sampled_nodes(workload, pair):
    """One FP64 step at the full workload size (the 256^3 D3Q27 + D3Q15 state,
    5.6 GB per buffer, takes the 64-bit addressing path) against the oracle
    at ~2000 sampled nodes."""
    print(f"workload={workload} pair={pair}", flush=True)
    cfg = workloads.config(workload, pair=pair)
    prm = params_from_config(cfg)
    lf, lg = prm.lattices
    wf = rest_weights(lf)
    wg = rest_weights(lg, thermal=True, cs2=prm.cs2T)
    sim = G.make_sim(cfg, "f64")
    S = G.full_hashed_state(cfg["shape"], lf.Q, lg.Q, wf, wg, seed=23, device="cuda")
    sim.import_fp64(S)
    del S
    sim.step(1)
    out = sim.export_fp64()
    x, y, z = G.sample_nodes(cfg["shape"], 2000, seed=24)
    got = out[:, z.cuda(), y.cuda(), x.cuda()].cpu()
    del out
    gf, gg = G.hashed_state_getters(cfg["shape"], lf.Q, lg.Q, wf, wg, seed=23)
    fo, go, _ = osim.step_at(prm, gf, gg, (x, y, z))
    assert G.rel_err(got[: lf.Q], fo) < 1e-13
    assert G.rel_err(got[lf.Q:], go) < 1e-13
    sim.close()


def test_fp_outlasts_mcm_in_the_sheared_cube():
    """The stability claim of Sec. 7 at one point of the Ma = 0.25, Pr = 0.71
    sweep on a 32^3 grid (D3Q27 + D3Q15, FP64): at Pe = 900 the FP model runs
    20,000 steps with the watchdog quiet, the MCM comparator trips it.  (The
    full sweep, ``python -m paper_2504_09041_amd.stability``, finds the largest
    stable Pe there at ~1,180 for FP and ~690 for MCM over 200,000 steps.)"""
    from paper_2504_09041_amd.stability import survives

    ok_fp, n_fp = survives("FP", 32, 0.25, 0.71, 900.0, 20000)
    ok_mcm, n_mcm = survives("MCM", 32, 0.25, 0.71, 900.0, 20000)
    print(f"FP: {ok_fp} ({n_fp} steps), MCM: {ok_mcm} ({n_mcm} steps)")
    assert ok_fp and not ok_mcm
