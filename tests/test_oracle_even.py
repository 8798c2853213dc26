"""Pins for oracle.even (GaNi on general grids, Sec. 4.4 and 5.2).

E1 the two triples {G^U, G^E_{N,0}, G^J_{N,I}} and {G^U, G^E_{N,I}, G^J_{N,0}} resolve
   the identity with mutually orthogonal projections (Lemma matrix_orthogonality_E).
E2 Proposition FD_even_problem: A_{H,N} = Btilde^-1 and B_{H,N}^-1 = Atilde on even
   grids, with B_{H,N}^-1 <= A_{H,N}; the gap is nonzero on even grids.
E3 odd grids reduce to oracle/gani.py; homogeneous media give A0 on any grid.
E4 the exact bounds of the minimisers enclose the Ga bounds of the same space Z_N^r.
E5 the paper's own bound values for the open square at contrast 1e3 on the grid 1024.
"""
import numpy as np
import pytest

import homgen
from oracle import even, galerkin as ga, gani, spectral as sp


def _square(rho, half=0.75):
    c = homgen.Inclusions(d=2, Y=np.array([2.0, 2.0]), A0=np.eye(2))
    c.add("rect", [0.0, 0.0], [2 * half, 2 * half], (1.0 + rho) * np.eye(2))
    return c


def _pix(seed=4, P=8):
    rng = np.random.default_rng(seed)
    return homgen.Pixels(d=2, Y=np.array([1.0, 1.3]), phase=(rng.random((P, P)) < 0.5).astype(np.int64),
                         phase_A=np.stack([np.eye(2), np.array([[8.0, 1.0], [1.0, 3.0]])]))


@pytest.mark.parametrize("shape", [(8, 8), (6, 9), (4, 6, 5)])
def test_E1_projection_triples(shape):
    d = len(shape)
    Y = np.array([1.0, 1.3, 0.8][:d])
    GE0, GEI, GJ0, GJI = even.projections(shape, Y)
    GU = sp.proj_U(shape) if all(n % 2 for n in shape) else _proj_U(shape)
    I = np.eye(d).reshape((d, d) + (1,) * d)
    mm = lambda A, B: np.einsum("ab...,bc...->ac...", A, B)
    for a, b, c in ((GU, GE0, GJI), (GU, GEI, GJ0)):
        assert np.abs(a + b + c - I).max() < 1e-13
        for P in (a, b, c):
            assert np.abs(mm(P, P) - P).max() < 1e-13
        for P, Q in ((a, b), (a, c), (b, c)):
            assert np.abs(mm(P, Q)).max() < 1e-13
    assert even.nyquist_mask(shape).any() == any(n % 2 == 0 for n in shape)


def _proj_U(shape):
    d = len(shape)
    G = np.zeros((d, d) + tuple(shape))
    G[(slice(None), slice(None)) + (0,) * d] = np.eye(d)
    return G


@pytest.mark.parametrize("case", ["S1_N8", "S2_N8", "pix_N8", "S1_N16_rho1e3"])
def test_E2_even_grid_duality(case):
    cell, N, closed = {"S1_N8": (_square(10.0), (8, 8), False), "S2_N8": (_square(10.0), (8, 8), True),
                       "pix_N8": (_pix(), (8, 8), False), "S1_N16_rho1e3": (_square(1e3), (16, 16), False)}[case]
    r = even.gani_general(cell, N, tol=1e-12, closed=closed)
    n = np.linalg.norm(r["A_HN"], 2)
    assert np.abs(r["A_HN"] - np.linalg.inv(r["B_tilde"])).max() <= 1e-9 * n
    assert np.abs(np.linalg.inv(r["B_HN"]) - r["A_tilde"]).max() <= 1e-9 * n
    gap = np.linalg.eigvalsh(r["A_HN"] - np.linalg.inv(r["B_HN"]))
    assert gap.min() >= -1e-10 * n and gap.max() > 1e-6 * n


def test_E2_open_and_closed_squares_differ_on_even_grids():
    # N = 8 on (-1, 1): grid points at multiples of 1/4, so x_a = +-3/4 lies on the interface
    a = even.gani_general(_square(10.0), (8, 8), closed=False, tilde=False)["A_HN"]
    b = even.gani_general(_square(10.0), (8, 8), closed=True, tilde=False)["A_HN"]
    assert b[0, 0] > a[0, 0] + 1e-3


@pytest.mark.parametrize("N", [(9, 9), (7, 11)])
def test_E3_odd_grids_reduce_to_gani(N):
    cell = _pix(P=7)
    r = even.gani_general(cell, N, tol=1e-12, tilde=False)
    g = gani.gani_bounds(cell, N, tol=1e-12)
    for k in ("A_HN", "B_HN", "A_up", "A_low"):
        assert np.abs(r[k] - g[k]).max() <= 1e-10 * np.linalg.norm(g[k], 2), k


def test_E3_homogeneous_on_even_grid():
    A0 = np.array([[3.0, 0.5], [0.5, 2.0]])
    cell = homgen.Inclusions(d=2, Y=np.array([1.0, 2.0]), A0=A0)
    r = even.gani_general(cell, (8, 6), tol=1e-13)
    for k in ("A_HN", "A_tilde", "A_up", "A_low"):
        assert np.abs(r[k] - A0).max() <= 1e-12, k
    assert np.abs(np.linalg.inv(r["B_HN"]) - A0).max() <= 1e-12


def test_E4_exact_bounds_enclose_the_ga_bounds_of_the_reduced_space():
    cell = _square(10.0)
    r = even.gani_general(cell, (16, 16), tol=1e-12, tilde=False)
    g = ga.bounds(ga.make_problem(cell, (15, 15)), tol=1e-12)
    n = np.linalg.norm(g["A_up"], 2)
    assert np.linalg.eigvalsh(r["A_up"] - g["A_up"]).min() >= -1e-10 * n
    assert np.linalg.eigvalsh(g["A_low"] - r["A_low"]).min() >= -1e-10 * n


def test_E5_paper_values_on_the_grid_1024():
    """The paper's own numbers (tests/golden/paper_even_grid_bounds.json): the
    upper and lower bounds of the GaNi minimisers of the open square S1 at
    contrast 1e3 on the grid 1024, with the paper's residual criterion 1e-8
    (remark on convergence criteria).  About two minutes on the CPU."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_even_grid_bounds.json")))
    n = gold["grid"]
    r = even.gani_general(_square(1e3), (n, n), tol=gold["residual_tolerance"], closed=False, tilde=False)
    ref = gold["values"]["S1"]
    assert abs(r["A_up"][0, 0] - ref["A_up"]) <= 1e-8 * ref["A_up"]
    assert abs(r["A_low"][0, 0] - ref["A_low"]) <= 1e-8 * ref["A_low"]
