"""Gradients through the FP central-moment LBM by its discrete adjoint.

The reverse sweep runs the hand-written adjoint kernels of ``libfpclbm.so``
(``fpc_adjoint_step``, ``fpc_adjoint_init``) over states recomputed from
checkpoints:

* forward: S_0 = init(T_init), S_n = Phi(S_{n-1}); the state is saved every
  K steps (device memory);
* backward, segment by segment from the last: restore the segment's first
  state, recompute and keep the segment's states, then apply the adjoint step
  from the segment's last step down to its first; finally the adjoint of the
  initial collision gives dJ/dT_init.  Memory: N/K checkpoints + K states.

The adjoint travels between steps as mu_n, the adjoint of the pulled
populations that enter the collision of step n + 1 (mu_N = 0); the kernels
apply the transpose of the pull when they read it.

Objectives are sums over time levels n of affine-in-T wall terms and kinetic
energies of the time-n macros:

* ``WallNusselt(face, n0, n1)``: mean over n in [n0, n1] of the wall Nusselt
  number <Nu>_face(n) of the one-sided stencil of Sec. 6.1; the library
  accumulates it during the forward steps and writes its adjoint seeds;
* ``KineticEnergy(n)``: 1/2 sum rho |u|^2 at time level n.

Gradients are with respect to a per-node Dirichlet wall-temperature profile
(``theta``) and the initial temperature field (``T_init``).
``ObjectiveFunction`` wraps a solver as a ``torch.autograd.Function``.
"""

from __future__ import annotations

import ctypes

import torch

from . import _abi as A
from .sim import FACE_INDEX, Simulation


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class WallNusselt:
    """Mean wall Nusselt number on ``face`` over time levels n0..n1 (inclusive).

    Its value accumulates on the device during the forward run
    (``fpc_step_nusselt``); its adjoint seeds come from ``fpc_nusselt_seed``."""

    def __init__(self, face, n0, n1):
        self.face = FACE_INDEX.get(face, face)
        self.n0, self.n1 = int(n0), int(n1)
        self._w = None
        self.direct_wall = 0.0

    def bind(self, sim):
        W = self.n1 - self.n0 + 1
        self._w, dTw = sim.nusselt_seed(self.face, 1.0 / W)
        # the wall term enters each of the W levels with weight 1 / W
        self.direct_wall = dTw * W

    def seed(self, n):
        if self.n0 <= n <= self.n1:
            return self._w, 0.0
        return None, 0.0

    def start(self, sim):
        """Term of time level 0 (host value)."""
        if self.n0 <= 0 <= self.n1:
            return sim.diagnostics(self.face)["nu"] / (self.n1 - self.n0 + 1)
        return 0.0

    def advance(self, sim, n, m, acc):
        """Step from level n to level m, adding the terms of levels n+1..m to
        acc (device); returns the host part (none)."""
        lo, hi = max(n + 1, self.n0), min(m, self.n1)
        if lo > hi:
            sim.step(m - n)
            return 0.0
        sim.step(lo - 1 - n)
        sim.step_nusselt(hi - lo + 1, self.face, 1.0 / (self.n1 - self.n0 + 1), acc)
        sim.step(m - hi)
        return 0.0


class KineticEnergy:
    """1/2 sum rho |u|^2 at time level n."""

    def __init__(self, n):
        self.n = int(n)
        self.direct_wall = 0.0
        self.face = -1

    def bind(self, sim):
        pass

    def seed(self, n):
        return (None, 1.0) if n == self.n else (None, 0.0)

    def start(self, sim):
        return sim.diagnostics(-1)["ke"] if self.n == 0 else 0.0

    def advance(self, sim, n, m, acc):
        if not n < self.n <= m:
            sim.step(m - n)
            return 0.0
        # the kernel of the step to level self.n also reduces KE over the
        # state it writes (no second pass over the state)
        v = float(sim.step_diagnostics(self.n - n, -1)[1].item())
        sim.step(m - self.n)
        return v


class AdjointSolver:
    """Forward run + checkpointed adjoint sweep for one objective.

    ``params``: fpc_params of the simulation; ``theta_face``: face whose
    Dirichlet temperature is the per-node profile ``theta`` (or None);
    ``nsteps``: N; ``every``: checkpoint interval K.
    """

    def __init__(self, params, nsteps, every, objective, theta_face=None, device=None):
        self.theta_face = FACE_INDEX.get(theta_face, theta_face) if theta_face is not None else None
        self.device = torch.device("cuda" if device is None else device)
        profiles = {}
        if self.theta_face is not None:
            k = self.theta_face // 2
            nx, ny, nz = params.nx, params.ny, params.nz
            shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[k]
            self.theta = torch.full(shp, float(params.wall_T[self.theta_face]), dtype=torch.float64,
                                    device=self.device)
            profiles[self.theta_face] = self.theta
        self.sim = Simulation(params, device=self.device, wall_profiles=profiles)
        if self.theta_face is not None:
            self.theta = self.sim._profiles[self.theta_face]
        self.N = int(nsteps)
        self.K = max(1, int(every))
        self.obj = objective
        self.obj.bind(self.sim)
        self.dt = torch.float64 if params.precision == A.FPC_FP64 else torch.float32
        self.ckpt = []
        self.T_init = None

    def forward(self, theta=None, T_init=None):
        sim = self.sim
        if theta is not None:
            self.theta.copy_(torch.as_tensor(theta, dtype=torch.float64).reshape(self.theta.shape))
        self.T_init = torch.as_tensor(T_init).to(self.device, torch.float64).contiguous().clone()
        sim.init(self.T_init)
        self.ckpt = [sim.save()]
        acc = torch.zeros(1, dtype=torch.float64, device=self.device)
        J = self.obj.start(sim)
        n = 0
        while n < self.N:
            m = min(n + self.K, self.N)
            J += self.obj.advance(sim, n, m, acc)
            n = m
            if n % self.K == 0 and n < self.N:
                self.ckpt.append(sim.save())
        return J + float(acc.item())

    def backward(self):
        """Returns (dJ/dtheta or None, dJ/dT_init)."""
        sim = self.sim
        lib = A.load()
        mu = sim.new_adjoint()  # mu_N = 0
        mu2 = sim.new_adjoint()
        dth = None
        ptrs = None
        if self.theta_face is not None:
            dth = torch.zeros_like(self.theta)
            arr = (ctypes.c_void_p * 6)()
            arr[self.theta_face] = dth.data_ptr()
            ptrs = arr
        # segment buffers, reused by every segment: the states S_{s0+1} ..
        # S_{s1-1} are rebuilt in place from the checkpoint S_{s0}
        seg = [sim.new_state() for _ in range(self.K - 1)]
        for s0 in reversed(range(0, self.N, self.K)):
            s1 = min(s0 + self.K, self.N)
            states = [self.ckpt[s0 // self.K]]
            for k in range(s1 - s0 - 1):
                sim.step_from(states[-1], seg[k])
                states.append(seg[k])
            for n in range(s1, s0, -1):
                w, ke = self.obj.seed(n)
                A.check(lib.fpc_adjoint_step(sim.handle, _ptr(states[n - 1 - s0]), _ptr(mu), _ptr(mu2),
                                             _ptr(w), ctypes.c_double(ke), ptrs), "fpc_adjoint_step")
                mu, mu2 = mu2, mu
            del states
        del seg
        w0, ke0 = self.obj.seed(0)
        dT = torch.empty_like(self.T_init)
        A.check(lib.fpc_adjoint_init(sim.handle, _ptr(self.T_init), _ptr(mu), _ptr(w0), ctypes.c_double(ke0),
                                     _ptr(dT)), "fpc_adjoint_init")
        if dth is not None and self.obj.face == self.theta_face:
            dth += self.obj.direct_wall.reshape(dth.shape)
        torch.cuda.synchronize(self.device)
        return dth, dT


class ObjectiveFunction(torch.autograd.Function):
    """J(theta, T_init) with gradients from the adjoint solver.

    ``J = ObjectiveFunction.apply(theta, T_init, solver)``.
    """

    @staticmethod
    def forward(ctx, theta, T_init, solver):
        J = solver.forward(theta.detach() if theta is not None else None, T_init.detach())
        ctx.solver = solver
        ctx.has_theta = theta is not None
        return torch.tensor(J, dtype=torch.float64, device=T_init.device)

    @staticmethod
    def backward(ctx, gJ):
        dth, dT = ctx.solver.backward()
        g = gJ.to(dT.device)
        return (g * dth if ctx.has_theta else None), g * dT, None
