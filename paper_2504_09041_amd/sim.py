"""Python front end of the C ABI: a simulation whose state lives in torch
device memory and whose kernels run on torch's current HIP stream.

Every step of the method runs in the HIP kernels of ``libfpclbm.so``; this
module only allocates buffers, marshals arguments and reshapes outputs.
"""

from __future__ import annotations

import ctypes

import torch

from . import _abi as A

FACE_INDEX = {"-x": 0, "+x": 1, "-y": 2, "+y": 3, "-z": 4, "+z": 5}
LATTICES = {"D2Q9-D2Q5": A.FPC_D2Q9_D2Q5, "D3Q27-D3Q7": A.FPC_D3Q27_D3Q7,
            "D2Q9-D2Q9": A.FPC_D2Q9_D2Q9, "D3Q27-D3Q15": A.FPC_D3Q27_D3Q15}
PRECISIONS = {"f64": A.FPC_FP64, "f32dev": A.FPC_FP32_DEV}
MODELS = {"FP": A.FPC_MODEL_FP, "MCM": A.FPC_MODEL_MCM}
THERMAL_OPTIONS = {"A": A.FPC_THERMAL_OPTION_A, "B": A.FPC_THERMAL_OPTION_B}
Q = {A.FPC_D2Q9_D2Q5: (9, 5, 2), A.FPC_D3Q27_D3Q7: (27, 7, 3), A.FPC_D2Q9_D2Q9: (9, 9, 2),
     A.FPC_D3Q27_D3Q15: (27, 15, 3)}


def face_code(fluid, thermal):
    if fluid == "periodic" or thermal == "periodic":
        if not (fluid == "periodic" and thermal == "periodic"):
            raise ValueError("a periodic face must be periodic for both distributions")
        return A.FPC_BC_PERIODIC
    table = {
        ("noslip", "adiabatic"): A.FPC_BC_NOSLIP_ADIABATIC,
        ("noslip", "dirichlet"): A.FPC_BC_NOSLIP_DIRICHLET,
        ("lid", "adiabatic"): A.FPC_BC_LID_ADIABATIC,
        ("lid", "dirichlet"): A.FPC_BC_LID_DIRICHLET,
    }
    return table[(fluid, thermal)]


def default_params(lattice, precision, shape):
    p = A.fpc_params()
    nx, ny, nz = shape
    A.call("fpc_params_default", ctypes.byref(p), LATTICES.get(lattice, lattice),
           PRECISIONS.get(precision, precision), nx, ny, nz)
    return p


def set_faces(p, faces):
    """faces: 6 dicts {fluid, thermal, T, u_w} in the order -x, +x, -y, +y, -z, +z."""
    for f, fd in enumerate(faces):
        p.bc[f] = face_code(fd["fluid"], fd["thermal"])
        p.wall_T[f] = float(fd.get("T", 0.0))
        for i, v in enumerate(fd.get("u_w", (0.0, 0.0, 0.0))):
            p.lid_u[f][i] = float(v)
    return p


def conduction_reference(p, axis):
    """Set the FP32-deviation thermal storage reference to the conduction
    profile between the two Dirichlet walls normal to ``axis`` (the library
    computes it from their wall temperatures)."""
    A.call("fpc_params_conduction_reference", ctypes.byref(p), int(axis))
    return p


def storage_reference(p):
    """(axis, slope) of the FP32 storage reference the parameters select
    (axis -1: the uniform T0)."""
    k = ctypes.c_int()
    s = ctypes.c_double()
    A.call("fpc_storage_reference", ctypes.byref(p), ctypes.byref(k), ctypes.byref(s))
    return k.value, s.value


def params_from_workload(cfg, precision="f64", shape=None, cs2_T=None, T_reference="auto", model="FP",
                         thermal_option="A"):
    """C parameters of a workload description (``workloads.CONFIGS`` entry).

    The physical -> lattice mapping runs in the library
    (fpc_params_natural / fpc_params_mixed).  ``T_reference`` picks the
    FP32-deviation storage reference of g: "auto" (the library's default: the
    conduction profile between the walls of a Dirichlet pair, else T0),
    "uniform" (T0) or "conduction" (between the Dirichlet walls normal to the
    workload's L axis).
    ``model``: "FP" or "MCM" (the Maxwellian comparator); ``thermal_option``:
    "A" or "B" (acts on the D2Q9 / D3Q15 thermal lattices)."""
    shape = tuple(cfg["shape"]) if shape is None else tuple(shape)
    p = default_params(cfg["pair"], precision, shape)
    p.model = MODELS[model]
    p.thermal_option = THERMAL_OPTIONS[thermal_option]
    if cs2_T is not None:
        p.cs2_T = float(cs2_T)
    if cfg["flow"] == "natural":
        A.call("fpc_params_natural", ctypes.byref(p), cfg["Ra"], cfg["Pr"], cfg["U0"], cfg["L_axis"],
               cfg["T_hot"], cfg["T_cold"])
    else:
        A.call("fpc_params_mixed", ctypes.byref(p), cfg["Re"], cfg["Ri"], cfg["Pe"], cfg["U_lid"],
               cfg["L_axis"], cfg["T_hot"], cfg["T_cold"])
    p.up_axis = cfg["up_axis"]
    set_faces(p, cfg["faces"])
    if T_reference == "conduction":
        conduction_reference(p, cfg["L_axis"])
    elif T_reference == "uniform":
        p.T_ref_axis = -1
        p.T_ref_slope = 0.0
    elif T_reference != "auto":
        raise ValueError("T_reference must be 'auto', 'uniform' or 'conduction'")
    return p


def state_bytes(p):
    """(bytes per state buffer, padded row length nxp) of the storage layout."""
    nb = ctypes.c_size_t()
    rs = ctypes.c_size_t()
    A.call("fpc_state_bytes", ctypes.byref(p), ctypes.byref(nb), ctypes.byref(rs))
    return nb.value, rs.value


class Simulation:
    """One FP central-moment thermal LBM simulation on a GPU."""

    def __init__(self, params, device=None, wall_profiles=None):
        if not torch.cuda.is_available():
            raise RuntimeError("Simulation needs a HIP GPU (torch.cuda is not available)")
        A.load()
        self.device = torch.device("cuda" if device is None else device)
        self.params = A.fpc_params()
        ctypes.memmove(ctypes.byref(self.params), ctypes.byref(params), ctypes.sizeof(params))
        self._profiles = {}
        for f, t in (wall_profiles or {}).items():
            fi = FACE_INDEX.get(f, f)
            t = t.to(self.device, torch.float64).contiguous()
            self._profiles[fi] = t
            self.params.wall_T_profile[fi] = t.data_ptr()
        self.nbytes, self.nxp = state_bytes(self.params)
        self.Qf, self.Qg, self.dim = Q[self.params.lattice]
        self.shape = (self.params.nx, self.params.ny, self.params.nz)
        self.N = self.params.nx * self.params.ny * self.params.nz
        self.Np = self.nxp * self.params.ny * self.params.nz  # padded node count
        self.dtype = torch.float64 if self.params.precision == A.FPC_FP64 else torch.float32
        with torch.cuda.device(self.device):
            self.buffers = [torch.empty(self.nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
            self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        A.call("fpc_create", ctypes.byref(self.params), self.buffers[0].data_ptr(), self.buffers[1].data_ptr(),
               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            A.call("fpc_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- stepping ----------------------------------------------------------
    def init(self, T_init):
        """T_init: (nz, ny, nx) temperature field (any device / dtype)."""
        T = torch.as_tensor(T_init).to(self.device, torch.float64).contiguous()
        if T.numel() != self.N:
            raise ValueError(f"T_init has {T.numel()} values, grid has {self.N}")
        self._tinit = T  # keep alive until the kernel has read it
        A.call("fpc_init", self._h, ctypes.c_void_p(T.data_ptr()))

    def step(self, n=1):
        A.call("fpc_step", self._h, int(n))

    def set_multistep(self, enable):
        """Allow (True, the default) or forbid fpc_step's single-launch
        multi-step path on small grids."""
        A.call("fpc_set_multistep", self._h, 1 if enable else 0)

    @property
    def multistep_launches(self):
        """Multi-step (cooperative) launches fpc_step has made so far."""
        v = ctypes.c_longlong()
        A.call("fpc_multistep_launches", self._h, ctypes.byref(v))
        return v.value

    def step_nusselt(self, n, face, weight, acc):
        """Advance n steps; after each, acc[0] += weight * <Nu>_face of the
        new time level (acc: one-element FP64 device tensor)."""
        if acc.dtype != torch.float64 or not acc.is_cuda or acc.numel() < 1:
            raise ValueError("acc must be a FP64 device tensor")
        A.call("fpc_step_nusselt", self._h, int(n), int(FACE_INDEX.get(face, face)), float(weight),
               ctypes.c_void_p(acc.data_ptr()))

    def step_diagnostics(self, n, face=-1, out=None):
        """Advance n >= 1 steps; the last step's kernel also reduces the
        diagnostics of the state it writes.  Returns the 5-element FP64 device
        tensor (nu, ke, sumT, umax, non-finite nodes) without synchronising."""
        if out is None:
            out = torch.empty(5, dtype=torch.float64, device=self.device)
        elif out.dtype != torch.float64 or not out.is_cuda or out.numel() < 5 or not out.is_contiguous():
            raise ValueError("out must be a contiguous FP64 device tensor of 5 elements")
        A.call("fpc_step_diagnostics", self._h, int(n), int(FACE_INDEX.get(face, face)),
               ctypes.c_void_p(out.data_ptr()))
        return out

    def nusselt_seed(self, face, weight=1.0):
        """Adjoint seeds of weight * <Nu>_face: (dJ/dT as an (nz, ny, nx)
        tensor, dJ/dT_w per wall node in the profile layout, flat)."""
        fi = FACE_INDEX.get(face, face)
        nx, ny, nz = self.shape
        M = self.N // (nx, ny, nz)[fi // 2]
        dT = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device)
        dTw = torch.empty(M, dtype=torch.float64, device=self.device)
        A.call("fpc_nusselt_seed", self._h, int(fi), float(weight), ctypes.c_void_p(dT.data_ptr()),
               ctypes.c_void_p(dTw.data_ptr()))
        return dT, dTw

    @property
    def step_count(self):
        v = ctypes.c_longlong()
        A.call("fpc_get_step", self._h, ctypes.byref(v))
        return v.value

    # -- outputs -----------------------------------------------------------
    def macros(self):
        nx, ny, nz = self.shape
        rho = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device)
        T = torch.empty_like(rho)
        u = torch.empty((self.dim, nz, ny, nx), dtype=torch.float64, device=self.device)
        A.call("fpc_macros", self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
               ctypes.c_void_p(T.data_ptr()))
        return {"rho": rho, "u": u, "T": T}

    def diagnostics(self, face=-1):
        """FP64 GPU reductions; returns dict(nu, ke, sumT, umax, unstable)."""
        fi = FACE_INDEX.get(face, face)
        vals = [ctypes.c_double() for _ in range(4)]
        rc = A.load().fpc_diagnostics(self._h, int(fi), *[ctypes.byref(v) for v in vals])
        if rc not in (A.FPC_OK, A.FPC_ERR_UNSTABLE):
            A.check(rc, "fpc_diagnostics")
        return {"nu": vals[0].value, "ke": vals[1].value, "sumT": vals[2].value, "umax": vals[3].value,
                "unstable": rc == A.FPC_ERR_UNSTABLE}

    def nusselt_local(self, face):
        """Local wall Nusselt numbers of the current time level on ``face``,
        shaped like the face's profile (slower tangential axis first)."""
        fi = FACE_INDEX.get(face, face)
        nx, ny, nz = self.shape
        shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[fi // 2]
        out = torch.empty(shp, dtype=torch.float64, device=self.device)
        A.call("fpc_nusselt_local", self._h, int(fi), ctypes.c_void_p(out.data_ptr()))
        return out

    def export_fp64(self):
        """Current state as full FP64 populations, shape (Qf + Qg, nz, ny, nx)."""
        nx, ny, nz = self.shape
        out = torch.empty((self.Qf + self.Qg, nz, ny, nx), dtype=torch.float64, device=self.device)
        A.call("fpc_export_fp64", self._h, ctypes.c_void_p(out.data_ptr()))
        return out

    def import_fp64(self, S, step=0):
        S = torch.as_tensor(S).to(self.device, torch.float64).contiguous()
        if S.numel() != (self.Qf + self.Qg) * self.N:
            raise ValueError("state has the wrong size")
        self._imp = S
        A.call("fpc_import_fp64", self._h, ctypes.c_void_p(S.data_ptr()), int(step))

    def save(self, out=None):
        if out is None:
            out = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        A.call("fpc_save", self._h, ctypes.c_void_p(out.data_ptr()))
        return out

    def new_state(self):
        """An uninitialised state buffer of this simulation's layout."""
        return torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)

    def step_from(self, src, dst):
        """dst = one step of src (caller-owned state buffers); the simulation's
        own state and step counter are untouched."""
        for b in (src, dst):
            if b.numel() != self.nbytes or b.dtype != torch.uint8 or not b.is_cuda:
                raise ValueError("state buffer has the wrong size, type or device")
        A.call("fpc_step_from", self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()))

    def load(self, buf, step=0):
        if buf.numel() != self.nbytes or buf.dtype != torch.uint8:
            raise ValueError("snapshot has the wrong size")
        A.call("fpc_load", self._h, ctypes.c_void_p(buf.data_ptr()), int(step))

    def current_buffer(self):
        p = ctypes.c_void_p()
        A.call("fpc_current_buffer", self._h, ctypes.byref(p))
        return p.value

    # -- storage layout ----------------------------------------------------
    # Rows are padded to nxp = nx rounded up to 64; tiles of 64 padded nodes
    # hold their Q populations as consecutive runs of 64 values (see
    # fpc_state_bytes in include/fpclbm.h).  These helpers only move values
    # between that layout and (Q, nz, ny, nx) arrays; padding is zero.
    def to_storage(self, values, dtype=None):
        """(Qf+Qg, nz, ny, nx) values -> flat tensor in the storage layout."""
        nx, ny, nz = self.shape
        Qt = self.Qf + self.Qg
        dt = self.dtype if dtype is None else dtype
        v = torch.as_tensor(values).to(self.device, dt).reshape(Qt, nz, ny, nx)
        pad = torch.zeros((Qt, nz, ny, self.nxp), dtype=dt, device=self.device)
        pad[..., :nx] = v
        return pad.reshape(Qt, self.Np // 64, 64).permute(1, 0, 2).contiguous().reshape(-1)

    def from_storage(self, buf):
        """Flat storage-layout tensor (elements, or the raw bytes of a state
        buffer) -> (Qf+Qg, nz, ny, nx) copy in its element type."""
        nx, ny, nz = self.shape
        Qt = self.Qf + self.Qg
        if buf.dtype == torch.uint8:
            buf = buf.view(self.dtype)
        t = buf.reshape(self.Np // 64, Qt, 64).permute(1, 0, 2).reshape(Qt, nz, ny, self.nxp)
        return t[..., :nx].contiguous()

    def new_adjoint(self):
        """A zeroed adjoint state (storage layout, the state's element type)."""
        return torch.zeros(self.Np * (self.Qf + self.Qg), dtype=self.dtype, device=self.device)

    def state_populations(self):
        """The current state in storage form (deviations in FP32_DEV mode),
        shape (Qf+Qg, nz, ny, nx)."""
        ptr = self.current_buffer()
        buf = self.buffers[0] if ptr == self.buffers[0].data_ptr() else self.buffers[1]
        return self.from_storage(buf)
