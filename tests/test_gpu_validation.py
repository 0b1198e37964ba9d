"""Physics self-validation against the paper's own FPC-LBM results.

The differentially heated square cavity is run to a steady state on the GPU
and its hot-wall Nusselt numbers are compared with the paper's printed values
(tests/golden/paper_cavity_nusselt.json, Sec. 6.1 Tables con2 and con3).  The
grids here are coarser than the paper's 512^2 and the thermal lattice is
D2Q5 (the paper's is D2Q9), so the bars are a physics check, not parity:
0.5 % on the mean Nusselt number and 1.5 % on its wall maximum and minimum.
The full-resolution runs (512^2, Ra 1e3-1e6, and the 128^3 cube) are made by
``python -m paper_2504_09041_amd.validate``.
"""

import json
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_cavity_nusselt.json")


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("key,n,U0", [("1e4", 128, 0.1), ("1e5", 256, 0.1)])
def test_cavity_nusselt_matches_paper(key, n, U0):
    from paper_2504_09041_amd.validate import cavity

    Ra = float(key)
    ref = json.load(open(GOLDEN))["2d"][key]
    print(f"Ra={Ra:g} n={n} U0={U0}", flush=True)
    r = cavity(2, Ra, n, U0=U0, chunk=10000, tol=1e-6, max_steps=2_000_000)
    print({k: r[k] for k in ("steps", "nu", "nu_max", "nu_min")})
    assert r["last_change"] < 1e-6
    assert abs(r["nu"] - ref["nu"]) <= 5e-3 * ref["nu"]
    assert abs(r["nu_max"] - ref["nu_max"]) <= 1.5e-2 * ref["nu_max"]
    assert abs(r["nu_min"] - ref["nu_min"]) <= 1.5e-2 * ref["nu_min"]
