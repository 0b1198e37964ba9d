"""Velocity sets and moment bases used by the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  Nothing under ``oracle/`` is part of the product:
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code, table or helper with the HIP
path in ``paper_2504_09041_amd``.

Sources (Schupbach & Premnath, "Fokker-Planck model based central moment
lattice Boltzmann method for effective simulations of thermal convective
flows", arXiv 2504.09041):

* D2Q9 velocity set, Eqs. (ex)/(ey) of Sec. 4.2; its ordered moment basis is
  the vector m^c listed right after those equations.
* D3Q27 velocity set and ordered moment basis, Sec. 5.2.
* D3Q15 velocity set and ordered moment basis, Sec. 5.4 (and App. C).
* D2Q5 / D3Q7 are not in the paper.  They are the axis-aligned subsets of
  D2Q9 / D3Q27 (the first five / seven vectors), with the moment basis cut to
  orders <= 2 along the axes.  This is the reading used for the thermal
  lattices of the hot path.

Each lattice also records how its diagonal second-order moments are grouped
for relaxation:

* 2D (App. A Step 3 for f, App. B Step 3 for g): the pair
  (k20 + k02, k20 - k02) is relaxed with rates (w3, w4).
* 3D fluid: the paper defers the D3Q27 rate assignment to its earlier work.
  The reading adopted here relaxes the trace k200+k020+k002 (bulk) and the two
  deviators k200-k020, k200-k002 (shear), which sit at the positions of
  k200, k020, k002 in the rate vector.
* 3D thermal (App. C Step 3): the three diagonal moments are relaxed one by
  one.
"""

from __future__ import annotations

import itertools

import torch

DT = torch.float64


class Lattice:
    """A discrete velocity set with its ordered list of moment exponents."""

    def __init__(self, name, vectors, moments, combo=None):
        self.name = name
        vecs = [tuple(int(c) for c in v) for v in vectors]
        self.d = len(vecs[0])
        self.Q = len(vecs)
        self.vectors = vecs
        self.E = torch.tensor(vecs, dtype=DT)  # (Q, d)
        self.M = [tuple(int(c) for c in m) for m in moments]
        if len(self.M) != self.Q:
            raise ValueError(f"{name}: {len(self.M)} moments for {self.Q} velocities")
        self.index = {m: k for k, m in enumerate(self.M)}
        self.opp = [vecs.index(tuple(-c for c in v)) for v in vecs]
        # combo = (positions of the grouped diagonal second-order moments, R)
        # with c = R @ kappa[positions]; None means no grouping.
        self.combo = combo

    def order(self, k):
        return sum(self.M[k])

    def __repr__(self):
        return f"Lattice({self.name})"


# --- D2Q9 (Eqs. ex, ey): rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1)
_EX_D2Q9 = (0, 1, 0, -1, 0, 1, -1, -1, 1)
_EY_D2Q9 = (0, 0, 1, 0, -1, 1, 1, -1, -1)
_M_D2Q9 = ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2))
_COMBO_2D = ((3, 4), ((1.0, 1.0), (1.0, -1.0)))

# --- D3Q27 (Sec. 5.2)
_EX_D3Q27 = (0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1)
_EY_D3Q27 = (0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1)
_EZ_D3Q27 = (0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1)
_M_D3Q27 = (
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2),
    (2, 0, 1), (0, 2, 1), (1, 1, 1), (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 1, 1),
    (1, 2, 1), (1, 1, 2), (1, 2, 2), (2, 1, 2), (2, 2, 1), (2, 2, 2),
)
_COMBO_3D_FLUID = ((7, 8, 9), ((1.0, 1.0, 1.0), (1.0, -1.0, 0.0), (1.0, 0.0, -1.0)))

# --- D3Q15 (Sec. 5.4)
_EX_D3Q15 = (0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1)
_EY_D3Q15 = (0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1)
_EZ_D3Q15 = (0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1)
_M_D3Q15 = (
    (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 2, 0), (0, 1, 2), (2, 0, 1), (1, 1, 1),
    (2, 2, 0),
)

D2Q9 = Lattice("D2Q9", list(zip(_EX_D2Q9, _EY_D2Q9)), _M_D2Q9, combo=_COMBO_2D)
D2Q9_T = Lattice("D2Q9-thermal", list(zip(_EX_D2Q9, _EY_D2Q9)), _M_D2Q9, combo=_COMBO_2D)
D2Q5 = Lattice(
    "D2Q5",
    list(zip(_EX_D2Q9[:5], _EY_D2Q9[:5])),
    ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2)),
    combo=_COMBO_2D,
)
D3Q27 = Lattice("D3Q27", list(zip(_EX_D3Q27, _EY_D3Q27, _EZ_D3Q27)), _M_D3Q27, combo=_COMBO_3D_FLUID)
D3Q7 = Lattice(
    "D3Q7",
    list(zip(_EX_D3Q27[:7], _EY_D3Q27[:7], _EZ_D3Q27[:7])),
    ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2)),
    combo=None,
)
D3Q15_T = Lattice("D3Q15-thermal", list(zip(_EX_D3Q15, _EY_D3Q15, _EZ_D3Q15)), _M_D3Q15, combo=None)

# Named pairs (fluid lattice, thermal lattice).  The first two are the hot
# path; the last two are the paper's own thermal lattices.
PAIRS = {
    "D2Q9-D2Q5": (D2Q9, D2Q5),
    "D3Q27-D3Q7": (D3Q27, D3Q7),
    "D2Q9-D2Q9": (D2Q9, D2Q9_T),
    "D3Q27-D3Q15": (D3Q27, D3Q15_T),
}


def full_tensor_product_set(d):
    """All vectors of {-1,0,1}^d (used by tests to check a velocity set)."""
    return set(itertools.product((-1, 0, 1), repeat=d))
