"""C-ABI checks that need no GPU: symbols, host-side validation, and the
library's physical -> lattice parameter mapping against the oracle's."""

import ctypes
import math
import os
import re

import pytest

import workloads
from oracle.params import params_from_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpclbm.h")

A = pytest.importorskip("paper_2504_09041_amd._abi")


def _lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libfpclbm.so not built")
    return A.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_names():
    assert declared_functions() == sorted(A.EXPORTED)


def test_build_compiles_every_hip_source():
    """Every HIP translation unit of the package is in the build (the adjoint
    kernels are split over several files that compile in parallel)."""
    from paper_2504_09041_amd import build as B

    on_disk = sorted(f for f in os.listdir(B.CSRC) if f.endswith(".hip"))
    assert sorted(B.SOURCES) == on_disk
    for f in ("fpc_adjoint.hip", "fpc_adjoint_d3q7.hip", "fpc_adjoint_d2q9.hip", "fpc_adjoint_d3q15.hip"):
        assert "-fno-honor-nans" in B.SOURCE_FLAGS[f]
    # the per-precision sources yield one object per precision, all named apart
    objs = [name for _, name, _ in B._units()]
    assert len(objs) == len(set(objs)) == len(B.SOURCES) + len(B.PER_PRECISION)
    for f in B.PER_PRECISION:
        text = open(os.path.join(B.CSRC, f)).read()
        assert "FPC_ADJ_REAL" in text


def _local_includes(csrc, name, seen):
    """Transitive closure of the package-local #include "..." of a source."""
    if name in seen:
        return seen
    seen.add(name)
    for inc in re.findall(r'^#include "([^"/]+)"', open(os.path.join(csrc, name)).read(), flags=re.M):
        _local_includes(csrc, inc, seen)
    return seen


@pytest.mark.parametrize("kind,roots", [("step", ["fpc_step.hip"]),
                                        ("adjoint", ["fpc_adjoint.hip", "fpc_adjoint_d3q7.hip"])])
def test_counter_records_match_the_kernel_sources(kind, roots):
    """The HBM-traffic records that the benchmark reports are fingerprinted by
    the kernel's sources: the fingerprint covers every file those sources
    include, and the committed records carry the fingerprint of the sources
    in the tree (they were taken on this code)."""
    import json

    import bench
    from paper_2504_09041_amd import build as B

    covered = set(bench.fingerprint_sources(kind))
    for root in roots:
        assert _local_includes(B.CSRC, root, set()) <= covered
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        records = json.load(fh)
    mine = [r for k, r in records.items() if k.startswith("adjoint_") == (kind == "adjoint")]
    assert mine
    for r in mine:
        assert r["sources"] == bench.kernel_fingerprint(kind)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.fpc_version() >= 10000


def test_params_struct_layout_matches_header():
    # offsets of the trailing members pin the struct layout used by ctypes
    p = A.fpc_params
    assert p.omega_f.offset == 20 + 4  # 5 ints, padded to 8
    assert p.T_ref_slope.offset == p.wall_T_profile.offset + 6 * 8
    assert p.T_ref_axis.offset == p.T_ref_slope.offset + 8
    assert p.model.offset == p.T_ref_axis.offset + 4
    assert p.thermal_option.offset == p.model.offset + 4
    assert ctypes.sizeof(p) == p.thermal_option.offset + 4 + 4  # padded to the struct's 8-byte alignment


def test_params_size_matches_library():
    lib = _lib()
    assert lib.fpc_params_bytes() == ctypes.sizeof(A.fpc_params)


def test_validation_errors():
    lib = _lib()
    p = A.fpc_params()
    assert lib.fpc_params_default(ctypes.byref(p), 7, 0, 8, 8, 1) == A.FPC_ERR_ARG
    assert lib.fpc_params_default(ctypes.byref(p), A.FPC_D2Q9_D2Q5, 0, 8, 8, 2) == A.FPC_ERR_SIZE
    assert lib.fpc_params_default(ctypes.byref(p), A.FPC_D2Q9_D2Q5, 0, 8, 8, 1) == A.FPC_OK
    nb, rs = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), ctypes.byref(rs)) == A.FPC_OK
    # rows padded to whole 64-node tiles: nxp = 64, 8 rows, Q = 14 FP64 values per node
    assert rs.value == 64 and nb.value == 64 * 8 * 14 * 8
    q = A.fpc_params()
    assert lib.fpc_params_default(ctypes.byref(q), A.FPC_D3Q27_D3Q7, A.FPC_FP32_DEV, 130, 3, 5) == A.FPC_OK
    assert lib.fpc_state_bytes(ctypes.byref(q), ctypes.byref(nb), ctypes.byref(rs)) == A.FPC_OK
    assert rs.value == 192 and nb.value == 192 * 3 * 5 * 34 * 4
    p.omega_f[4] = 2.0
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    assert "omega_f[4]" in A.last_error()
    p.omega_f[4] = 1.0
    p.bc[0] = A.FPC_BC_NOSLIP_ADIABATIC  # periodic on +x only
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.bc[1] = A.FPC_BC_LID_ADIABATIC
    p.lid_u[1][0] = 0.1  # normal component on an x face
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.lid_u[1][0] = 0.0
    p.lid_u[1][1] = 0.1
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_OK
    p.bc[4] = A.FPC_BC_NOSLIP_ADIABATIC
    p.bc[5] = A.FPC_BC_NOSLIP_ADIABATIC
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.bc[4] = p.bc[5] = A.FPC_BC_PERIODIC
    # thermal storage reference: axis in range, not periodic, finite slope
    assert p.T_ref_axis == A.FPC_TREF_AUTO and p.T_ref_slope == 0.0
    p.T_ref_slope = 0.01
    p.T_ref_axis = 2
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.T_ref_axis = 0  # x is walled by now
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_OK
    p.T_ref_axis = 1  # y is periodic
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.T_ref_axis = 0
    p.T_ref_slope = float("nan")
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
    p.T_ref_slope = 0.0
    h = ctypes.c_void_p()
    assert lib.fpc_create(None, None, None, None, ctypes.byref(h)) == A.FPC_ERR_ARG
    assert lib.fpc_step(None, 1) == A.FPC_ERR_ARG


@pytest.mark.parametrize("name", list(workloads.CONFIGS))
def test_parameter_mapping_matches_oracle(name):
    from paper_2504_09041_amd.sim import params_from_workload

    _lib()
    cfg = workloads.config(name)
    precs = ("f64",) if cfg["pair"] in ("D2Q9-D2Q9", "D3Q27-D3Q15") else ("f64", "f32dev")
    for prec in precs:
        p = params_from_workload(cfg, prec)
        o = params_from_config(cfg)
        lf, lg = o.lattices
        for k in range(1, lf.Q):
            assert math.isclose(p.omega_f[k], o.omega_f[k], rel_tol=1e-14), (k, p.omega_f[k], o.omega_f[k])
        for k in range(1, lg.Q):
            assert math.isclose(p.omega_g[k], o.omega_g[k], rel_tol=1e-14)
        assert math.isclose(p.g_beta, o.g_beta, rel_tol=1e-14)
        assert math.isclose(p.cs2_T, o.cs2T, rel_tol=1e-15)
        assert p.T0 == o.T0 and p.up_axis == o.up_axis


def test_storage_layout_helpers_match_the_documented_layout():
    """Simulation.to_storage / from_storage place population q of node
    (x, y, z) at element (t Q + q) 64 + n % 64, n = (z ny + y) nxp + x,
    t = n // 64 (the layout fpc_state_bytes documents), and round-trip."""
    import types

    import torch

    from paper_2504_09041_amd.sim import Simulation

    nx, ny, nz, Qf, Qg = 70, 3, 2, 9, 5
    nxp = 128
    m = types.SimpleNamespace(shape=(nx, ny, nz), Qf=Qf, Qg=Qg, nxp=nxp, Np=nxp * ny * nz,
                              dtype=torch.float64, device=torch.device("cpu"))
    Q = Qf + Qg
    vals = torch.arange(Q * nz * ny * nx, dtype=torch.float64).reshape(Q, nz, ny, nx) + 1.0
    flat = Simulation.to_storage(m, vals)
    assert flat.numel() == m.Np * Q
    for q, z, y, x in [(0, 0, 0, 0), (3, 1, 2, 69), (13, 0, 1, 64), (7, 1, 0, 63), (Qf, 1, 2, 5)]:
        n = (z * ny + y) * nxp + x
        assert flat[(n // 64 * Q + q) * 64 + n % 64] == vals[q, z, y, x]
    # padding nodes (x >= nx) are zero
    n = (1 * ny + 2) * nxp + 100
    assert flat[(n // 64 * Q + 2) * 64 + n % 64] == 0
    assert torch.equal(Simulation.from_storage(m, flat), vals)
    assert torch.equal(Simulation.from_storage(m, flat.view(torch.uint8)), vals)


@pytest.mark.parametrize("wl,shape", [("dhc2d_64", (1, 5, 1)), ("mixed2d_512", (5, 1, 1)),
                                      ("dhc3d_256", (4, 3, 1))])
def test_walled_axis_of_one_node_is_rejected(wl, shape):
    """A walled axis needs two nodes (the wall Nusselt stencil reads two
    layers): the library refuses one before any launch; a periodic axis of
    one node is accepted."""
    import workloads
    from paper_2504_09041_amd.sim import params_from_workload, state_bytes

    with pytest.raises(A.FpcError) as e:
        state_bytes(params_from_workload(workloads.config(wl, shape=shape), "f64"))
    assert e.value.code == A.FPC_ERR_SIZE
    nb, nxp = state_bytes(params_from_workload(workloads.config("rb2d_1024x512", shape=(1, 6, 1)), "f64"))
    assert nxp == 64 and nb == 64 * 6 * 14 * 8


def test_size_limits():
    """Largest grids: the padded node count nxp ny nz must stay below 2^31
    (32-bit node indices in the kernels) and a state below 4e10 populations;
    just below the limits is accepted."""
    lib = _lib()
    nb = ctypes.c_size_t()

    def state_rc(lattice, nx, ny, nz):
        p = A.fpc_params()
        assert lib.fpc_params_default(ctypes.byref(p), lattice, A.FPC_FP32_DEV, nx, ny, nz) == A.FPC_OK
        return lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None)

    # 2D: 65536 x 32767 padded nodes < 2^31
    assert state_rc(A.FPC_D2Q9_D2Q5, 65536, 32767, 1) == A.FPC_OK
    assert nb.value == 65536 * 32767 * 14 * 4
    # 65536 x 32768 = 2^31 padded nodes: rejected
    assert state_rc(A.FPC_D2Q9_D2Q5, 65536, 32768, 1) == A.FPC_ERR_SIZE
    # padding counts: nx = 65473 pads to 65536
    assert state_rc(A.FPC_D2Q9_D2Q5, 65473, 32768, 1) == A.FPC_ERR_SIZE
    # 3D: 1290^3 padded to 1344 x 1290 x 1290 > 2^31
    assert state_rc(A.FPC_D3Q27_D3Q7, 1290, 1290, 1290) == A.FPC_ERR_SIZE
    assert state_rc(A.FPC_D3Q27_D3Q7, 1024, 1024, 1024) == A.FPC_OK
    # more than 4e10 populations per state (1280^3 x 34) is rejected as well
    assert state_rc(A.FPC_D3Q27_D3Q7, 1280, 1280, 1280) == A.FPC_ERR_SIZE


def test_null_and_invalid_arguments_fail_before_any_launch():
    """Argument errors are caught on the host and reported through the status
    code and fpc_last_error, without touching a device."""
    lib = _lib()
    vp = ctypes.c_void_p
    p = A.fpc_params()
    assert lib.fpc_params_default(ctypes.byref(p), A.FPC_D2Q9_D2Q5, A.FPC_FP64, 8, 8, 1) == A.FPC_OK
    h = vp()
    # NULL parameters / output handle
    assert lib.fpc_create(None, vp(256), vp(512), None, ctypes.byref(h)) == A.FPC_ERR_ARG
    assert lib.fpc_create(ctypes.byref(p), vp(256), vp(512), None, None) == A.FPC_ERR_ARG
    # missing, identical or unaligned state buffers (never dereferenced)
    assert lib.fpc_create(ctypes.byref(p), None, vp(512), None, ctypes.byref(h)) == A.FPC_ERR_ARG
    assert lib.fpc_create(ctypes.byref(p), vp(256), vp(256), None, ctypes.byref(h)) == A.FPC_ERR_ARG
    assert lib.fpc_create(ctypes.byref(p), vp(256), vp(520), None, ctypes.byref(h)) == A.FPC_ERR_ARG
    assert "aligned" in A.last_error()
    assert h.value is None
    # invalid parameters are rejected by fpc_create as by fpc_state_bytes
    p.omega_f[4] = 0.0
    assert lib.fpc_create(ctypes.byref(p), vp(256), vp(512), None, ctypes.byref(h)) == A.FPC_ERR_ARG
    # NULL simulation handle on every call that takes one
    ll = ctypes.c_longlong()
    d = ctypes.c_double()
    assert lib.fpc_destroy(None) == A.FPC_ERR_ARG
    assert lib.fpc_set_stream(None, None) == A.FPC_ERR_ARG
    assert lib.fpc_set_multistep(None, 1) == A.FPC_ERR_ARG
    assert lib.fpc_set_multistep_wait_limit(None, 1) == A.FPC_ERR_ARG
    assert lib.fpc_multistep_launches(None, ctypes.byref(ll)) == A.FPC_ERR_ARG
    assert lib.fpc_init(None, vp(256)) == A.FPC_ERR_ARG
    assert lib.fpc_step(None, 1) == A.FPC_ERR_ARG
    assert lib.fpc_step_from(None, vp(256), vp(512)) == A.FPC_ERR_ARG
    assert lib.fpc_step_nusselt(None, 1, 2, ctypes.c_double(1.0), vp(256)) == A.FPC_ERR_ARG
    assert lib.fpc_step_diagnostics(None, 1, -1, vp(256)) == A.FPC_ERR_ARG
    assert lib.fpc_get_step(None, ctypes.byref(ll)) == A.FPC_ERR_ARG
    assert lib.fpc_macros(None, None, None, None) == A.FPC_ERR_ARG
    assert lib.fpc_diagnostics(None, 0, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d),
                               ctypes.byref(d)) == A.FPC_ERR_ARG
    assert lib.fpc_save(None, vp(256)) == A.FPC_ERR_ARG
    assert lib.fpc_load(None, vp(256), 0) == A.FPC_ERR_ARG
    assert lib.fpc_export_fp64(None, vp(256)) == A.FPC_ERR_ARG
    assert lib.fpc_import_fp64(None, vp(256), 0) == A.FPC_ERR_ARG
    assert lib.fpc_current_buffer(None, ctypes.byref(vp())) == A.FPC_ERR_ARG
    assert lib.fpc_adjoint_step(None, vp(256), vp(512), vp(768), None, ctypes.c_double(0.0), None) == A.FPC_ERR_ARG
    assert lib.fpc_adjoint_init(None, vp(256), vp(512), None, ctypes.c_double(0.0), vp(768)) == A.FPC_ERR_ARG
    assert "NULL" in A.last_error()
    # NULL parameter blocks of the helpers
    assert lib.fpc_params_default(None, A.FPC_D2Q9_D2Q5, A.FPC_FP64, 8, 8, 1) == A.FPC_ERR_ARG
    assert lib.fpc_params_natural(None, 1e6, 0.71, 0.05, 1, 0.5, -0.5) == A.FPC_ERR_ARG
    assert lib.fpc_params_mixed(None, 100.0, 1.0, 71.0, 0.1, 1, 0.5, -0.5) == A.FPC_ERR_ARG
    assert lib.fpc_state_bytes(None, None, None) == A.FPC_ERR_ARG


@pytest.mark.parametrize("name", ["dhc2d_64", "rb2d_1024x512", "dhc3d_256", "mixed2d_512", "rb3d_128"])
def test_default_storage_reference_is_the_conduction_profile(name):
    """FPC_TREF_AUTO resolves to the conduction profile between the
    workload's Dirichlet walls: axis L, slope (T_+ - T_-) / n_L, the line
    through the two wall temperatures with the walls halfway outside the
    outermost nodes (its values at x = -1/2 and n - 1/2 are the wall
    temperatures)."""
    from paper_2504_09041_amd.sim import params_from_workload, storage_reference

    _lib()
    cfg = workloads.config(name)
    k = cfg["L_axis"]
    n = cfg["shape"][k]
    lo, hi = cfg["faces"][2 * k]["T"], cfg["faces"][2 * k + 1]["T"]
    p = params_from_workload(cfg, "f32dev")
    assert p.T_ref_axis == A.FPC_TREF_AUTO
    axis, slope = storage_reference(p)
    assert axis == k
    T0 = p.T0
    assert abs((T0 + slope * (-0.5 - (n - 1) / 2)) - lo) < 1e-15
    assert abs((T0 + slope * (n - 0.5 - (n - 1) / 2)) - hi) < 1e-15
    # the explicit conduction reference is the same; uniform and FP64 report none
    assert storage_reference(params_from_workload(cfg, "f32dev", T_reference="conduction")) == (axis, slope)
    assert storage_reference(params_from_workload(cfg, "f32dev", T_reference="uniform")) == (-1, 0.0)
    assert storage_reference(params_from_workload(cfg, "f64")) == (-1, 0.0)


def test_storage_reference_choices_and_errors():
    from paper_2504_09041_amd.sim import params_from_workload, storage_reference

    lib = _lib()
    # no Dirichlet pair (adiabatic or periodic everywhere): the uniform reference
    cfg = workloads.config("dhc2d_64")
    cfg["faces"][0] = dict(cfg["faces"][2])
    cfg["faces"][1] = dict(cfg["faces"][2])
    p = params_from_workload(cfg, "f32dev")
    assert storage_reference(p) == (-1, 0.0)
    assert lib.fpc_params_conduction_reference(ctypes.byref(p), 0) == A.FPC_ERR_ARG
    assert lib.fpc_params_conduction_reference(ctypes.byref(p), 2) == A.FPC_ERR_ARG
    # two Dirichlet pairs: the larger wall-temperature difference wins
    cfg = workloads.config("dhc3d_256", shape=(8, 6, 10))
    cfg["faces"][4] = {"fluid": "noslip", "thermal": "dirichlet", "T": 2.0, "u_w": (0.0, 0.0, 0.0)}
    cfg["faces"][5] = {"fluid": "noslip", "thermal": "dirichlet", "T": -1.0, "u_w": (0.0, 0.0, 0.0)}
    p = params_from_workload(cfg, "f32dev")
    assert storage_reference(p) == (2, -3.0 / 10)
    assert lib.fpc_params_conduction_reference(ctypes.byref(p), 0) == A.FPC_OK
    assert storage_reference(p) == (0, -1.0 / 8)
    p.T_ref_axis = -3
    nb = ctypes.c_size_t()
    assert lib.fpc_state_bytes(ctypes.byref(p), ctypes.byref(nb), None) == A.FPC_ERR_ARG
