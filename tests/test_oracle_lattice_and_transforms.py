"""Pins of the oracle's lattices, weights and moment transforms (CPU only).

Each check compares the oracle with something it does not compute itself:
textbook lattice weights, the complete {-1,0,1}^d velocity sets, the
paper's printed App. A matrices P and P^-1 (golden fixture), and the frame
transform F(u) written as the binomial expansion Sec. 4.2 describes.
"""

import itertools

import pytest
import torch

from oracle import lattices as L
from oracle.collision import cm_matrix, raw_matrix, rest_weights
from tests import cm_binomial_2d as B

DT = torch.float64


def test_velocity_sets():
    assert set(L.D2Q9.vectors) == L.full_tensor_product_set(2)
    assert set(L.D3Q27.vectors) == L.full_tensor_product_set(3)
    axes3 = {(0, 0, 0)} | {tuple(s if i == k else 0 for i in range(3)) for k in range(3) for s in (-1, 1)}
    assert set(L.D3Q7.vectors) == axes3
    axes2 = {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)}
    assert set(L.D2Q5.vectors) == axes2
    corners = set(itertools.product((-1, 1), repeat=3))
    assert set(L.D3Q15_T.vectors) == axes3 | corners
    for lat in (L.D2Q9, L.D2Q5, L.D3Q27, L.D3Q7, L.D3Q15_T):
        assert len(set(lat.vectors)) == lat.Q
        for a in range(lat.Q):
            assert lat.vectors[lat.opp[a]] == tuple(-c for c in lat.vectors[a])
    # D3Q27 moment basis: every exponent combination in {0,1,2}^3 exactly once
    assert set(L.D3Q27.M) == set(itertools.product((0, 1, 2), repeat=3))


@pytest.mark.parametrize(
    "lat,thermal,cs2,expected",
    [
        (L.D2Q9, False, 1 / 3, {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}),
        (L.D3Q27, False, 1 / 3, {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}),
        (L.D3Q15_T, True, 1 / 3, {0: 2 / 9, 1: 1 / 9, 3: 1 / 72}),
        (L.D2Q5, True, 1 / 3, {0: 1 / 3, 1: 1 / 6}),
        (L.D3Q7, True, 0.25, {0: 0.25, 1: 0.125}),
        (L.D3Q7, True, 1 / 3, {0: 0.0, 1: 1 / 6}),
    ],
)
def test_rest_weights_textbook(lat, thermal, cs2, expected):
    """Lattice weights (standard values; D2Q5/D3Q7: 1 - d c^2, c^2/2)."""
    w = rest_weights(lat, thermal=thermal, cs2=cs2)
    for a, v in enumerate(lat.vectors):
        n1 = sum(abs(c) for c in v)
        assert abs(float(w[a]) - expected[n1]) < 1e-15, (lat.name, a)
    assert abs(float(w.sum()) - 1.0) < 1e-15


def test_raw_matrix_and_inverse_match_appendix_A():
    """P (App. A Step 1) and P^-1 (App. A Step 5) for D2Q9, as printed."""
    P = raw_matrix(L.D2Q9)
    Pp, Pinv = B.printed_matrices()
    assert torch.equal(P, Pp)
    assert torch.allclose(torch.linalg.inv(P), Pinv, atol=1e-15, rtol=0)


def test_frame_transform_is_the_binomial_shift():
    """C(u) f equals the raw moments shifted by -u with binomial coefficients
    (F(u) of Sec. 4.2), and the +u shift takes the central moments back."""
    g = torch.Generator().manual_seed(7)
    u = (torch.rand(50, 2, generator=g, dtype=DT) - 0.5) * 0.6
    f = torch.rand(50, 9, generator=g, dtype=DT)
    C = cm_matrix(L.D2Q9, u)
    kap = torch.einsum("nkq,nq->nk", C, f)
    raw = B.raw_moments(f)
    kp = B.shift(raw, u[:, 0], u[:, 1], -1)
    assert torch.allclose(kap, torch.stack([kp[m] for m in B.ORDER], 1), atol=1e-14, rtol=0)
    back = B.shift({m: kap[:, i] for i, m in enumerate(B.ORDER)}, u[:, 0], u[:, 1], +1)
    for m in B.ORDER:
        assert torch.allclose(back[m], raw[m], atol=1e-14, rtol=0)
    # and the printed P^-1 recovers the populations from the raw moments
    assert torch.allclose(B.populations(raw), f, atol=1e-14, rtol=0)


@pytest.mark.parametrize("lat", [L.D2Q9, L.D2Q5, L.D3Q27, L.D3Q7])
def test_inverse_frame_is_negated_velocity(lat):
    """On these lattices F^-1(u) = F(-u), i.e. C(u)^-1 = P^-1 F(-u)."""
    g = torch.Generator().manual_seed(11)
    u = (torch.rand(20, lat.d, generator=g, dtype=DT) - 0.5) * 0.6
    P = raw_matrix(lat)
    Fu = cm_matrix(lat, u) @ torch.linalg.inv(P)
    Fm = cm_matrix(lat, -u) @ torch.linalg.inv(P)
    eye = torch.eye(lat.Q, dtype=DT).expand(20, -1, -1)
    assert torch.allclose(Fu @ Fm, eye, atol=1e-13, rtol=0)


def test_d3q15_frame_is_not_negated_velocity():
    """D3Q15 aliases e_x^2 e_y with e_y e_z^2, so its F^-1(u) differs from F(-u)."""
    u = torch.tensor([[0.1, -0.2, 0.15]], dtype=DT)
    P = raw_matrix(L.D3Q15_T)
    Fu = cm_matrix(L.D3Q15_T, u) @ torch.linalg.inv(P)
    Fm = cm_matrix(L.D3Q15_T, -u) @ torch.linalg.inv(P)
    assert (Fu @ Fm - torch.eye(15, dtype=DT)).abs().max() > 1e-3


@pytest.mark.parametrize("name,lat", [("D2Q9", L.D2Q9), ("D3Q27", L.D3Q27), ("D3Q15", L.D3Q15_T)])
def test_orderings_match_the_printed_ones(name, lat):
    """Velocity and moment orders as printed (Sec. 4.2, 5.2, 5.4): the moment
    order is the order of the relaxation-rate slots."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_lattice_orderings.json")
    with open(path) as fh:
        ref = json.load(fh)[name]
    comps = [ref[k] for k in ("ex", "ey", "ez") if k in ref]
    assert lat.vectors == [tuple(c[a] for c in comps) for a in range(lat.Q)]
    assert lat.M == [tuple(int(ch) for ch in m) for m in ref["moments"]]
    # the thermal axis lattices are the leading vectors of the fluid ones
    if name == "D2Q9":
        assert L.D2Q5.vectors == lat.vectors[:5]
    if name == "D3Q27":
        assert L.D3Q7.vectors == lat.vectors[:7]
