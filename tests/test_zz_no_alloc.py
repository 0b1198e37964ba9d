"""fpc_diagnostics_noalloc (through the C ABI) against fpc_diagnostics.

The allocation-free entry point runs the same reduction kernels with the
library's static device scratch instead of the simulation's allocated one,
and writes its results to caller-owned device memory without synchronising.
Both use the same summation order, so the values must be bit-identical.  Two
calls in a row on one GPU, the second on a smaller grid, check that the
shared scratch carries nothing over from the previous call.
"""

import ctypes

import pytest
import torch

import workloads
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    G.need_gpu()


CALLS = [
    # (workload, shape, precision): a grid large enough that the node
    # reduction strides (more than 1024 blocks of 256 nodes), then a smaller one
    ("dhc3d_256", (128, 64, 48), "f32dev"),
    ("rb2d_1024x512", (50, 20, 1), "f64"),
]


def test_noalloc_diagnostics_equal_fpc_diagnostics():
    from paper_2504_09041_amd import _abi as A

    lib = A.load()
    for wl, shape, precision in CALLS:
        print(f"noalloc diagnostics: {wl} {shape} {precision}", flush=True)
        cfg = workloads.config(wl, shape=shape)
        sim = G.make_sim(cfg, precision)
        T = G.initial_T(cfg) + 0.05 * torch.tensor(workloads.uniform_field(tuple(shape[::-1]), 3))
        sim.init(T.cuda())
        sim.step(20)
        for face in (cfg["nu_face"], -1):
            out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
            A.check(lib.fpc_diagnostics_noalloc(sim.handle, face, ctypes.c_void_p(out.data_ptr())),
                    "fpc_diagnostics_noalloc")
            torch.cuda.synchronize()
            got = out.cpu().tolist()
            ref = sim.diagnostics(face)
            assert got[0] == (ref["nu"] if face >= 0 else 0.0)
            assert got[1] == ref["ke"]
            assert got[2] == ref["sumT"]
            assert got[3] == ref["umax"]
            assert got[4] == 0.0
            assert ref["ke"] > 0.0 and ref["umax"] > 0.0
        sim.close()


def test_noalloc_diagnostics_rejects_bad_arguments():
    from paper_2504_09041_amd import _abi as A

    lib = A.load()
    cfg = workloads.config("rb2d_1024x512", shape=(16, 8, 1))
    sim = G.make_sim(cfg, "f64")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(out.data_ptr())
    assert lib.fpc_diagnostics_noalloc(None, 2, p) == A.FPC_ERR_ARG
    assert lib.fpc_diagnostics_noalloc(sim.handle, 2, None) == A.FPC_ERR_ARG
    assert lib.fpc_diagnostics_noalloc(sim.handle, 7, p) == A.FPC_ERR_ARG
    assert lib.fpc_diagnostics_noalloc(sim.handle, 0, p) == A.FPC_ERR_STATE  # periodic x face
    assert lib.fpc_diagnostics_noalloc(sim.handle, 4, p) == A.FPC_ERR_STATE  # 2D has no z faces
    sim.close()
