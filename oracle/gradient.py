"""Reference objectives for gradient checks, differentiated by torch autograd.

TEST INFRASTRUCTURE ONLY (see ``oracle/lattices.py``).

The objectives are evaluated on the oracle's own time stepping (FP64, CPU),
so their autograd gradients are the reference for the hand-written adjoint of
the HIP path:

* wall Nusselt number averaged over time levels n0..n1 (the one-sided wall
  stencil of Sec. 6.1, on the time-n temperature);
* kinetic energy 1/2 sum rho |u|^2 at one time level n.
"""

from __future__ import annotations

import torch

from . import sim as osim


def objective(prm, T_init, nsteps, kind, face=None, window=None, theta_face=None, theta=None, at=None):
    """J for the run S_0 = init(T_init), S_n = step(S_{n-1}), n = 1..nsteps."""
    wall_T = {theta_face: theta} if theta_face is not None else None
    f, g = osim.init_state(prm, T_init)
    J = torch.zeros((), dtype=torch.float64)
    for n in range(1, nsteps + 1):
        f, g, mac = osim.step(prm, f, g, wall_T)
        if kind == "nu" and window[0] <= n <= window[1]:
            J = J + osim.nusselt(prm, mac["T"], face, wall_T) / (window[1] - window[0] + 1)
        if kind == "ke" and n == at:
            J = J + osim.kinetic_energy(mac)
    return J


def gradient(prm, T_init, nsteps, kind, face=None, window=None, theta_face=None, theta=None, at=None):
    """(J, dJ/dtheta or None, dJ/dT_init) by reverse-mode autograd."""
    T = T_init.detach().clone().requires_grad_(True)
    th = theta.detach().clone().requires_grad_(True) if theta is not None else None
    J = objective(prm, T, nsteps, kind, face, window, theta_face, th, at)
    inputs = [T] + ([th] if th is not None else [])
    grads = torch.autograd.grad(J, inputs, allow_unused=True)
    gT = grads[0] if grads[0] is not None else torch.zeros_like(T)
    gth = None
    if th is not None:
        gth = grads[1] if grads[1] is not None else torch.zeros_like(th)
    return float(J.detach()), gth, gT
