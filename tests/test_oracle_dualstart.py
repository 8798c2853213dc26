"""Pins for oracle.dualstart (Proposition FD_odd_problem (ii), eq.
FD_superposition_odd_A, and the remark on avoiding the dual solution).

D1 GaNi on odd grids: the start from converged primal minimisers equals the
   dual GaNi minimiser, with or without the projection (the superposition is
   already in J_N when the primal minimisers are exact).
D2 Ga: the start lies in J_N (G^J leaves it unchanged), its dual energy is at
   least the converged one and far below the zero start's, and CG from it
   reaches the converged bounds.
"""
import numpy as np
import pytest

import homgen
from oracle import coefficients as co, dualstart as ds, galerkin as ga, gani, spectral as sp


def _aniso_rects(seed=3):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


CELLS = [
    ("pix", lambda: homgen.pixel_cell(seed=21, P=9, values=(1.0, 20.0)), (9, 9)),
    ("aniso", _aniso_rects, (9, 15)),
    ("sph3d", lambda: homgen.sphere_cell(seed=22, n=3, anisotropic=True), (5, 7, 5)),
]


@pytest.mark.parametrize("name,make,N", CELLS, ids=[c[0] for c in CELLS])
def test_D1_gani_start_is_the_dual_minimiser(name, make, N):
    cell = make()
    d = cell.d
    Y = np.asarray(cell.Y, float)
    AN = co.point_values(cell, N)
    I = np.eye(d)
    xs = [gani.gani_solve(AN, N, Y, I[a], tol=1e-13)[0] for a in range(d)]
    js = [gani.gani_solve(AN, N, Y, I[a], dual=True, tol=1e-13)[0] for a in range(d)]
    # A_{H,N} by the trapezoidal energy of the primal minimisers
    A_HN = np.array([[np.mean(np.sum((xs[b] + I[b].reshape((d,) + (1,) * d)) *
                                     np.einsum("ij...,j...->i...", AN, xs[a] + I[a].reshape((d,) + (1,) * d)),
                                     axis=0)) for b in range(d)] for a in range(d)])
    for project in (True, False):
        st = ds.gani_dual_start(AN, Y, xs, A_HN, project=project)
        for b in range(d):
            scale = np.abs(js[b]).max() + 1.0
            assert np.abs(st[b] - js[b]).max() <= 1e-9 * scale, (project, b)


@pytest.mark.parametrize("name,make,N", CELLS[:2], ids=[c[0] for c in CELLS[:2]])
def test_D2_ga_start_is_admissible_and_close(name, make, N):
    cell = make()
    d = cell.d
    prob = ga.make_problem(cell, N)
    ref = ga.bounds(prob, tol=1e-12)
    I = np.eye(d)
    prim = [ga.solve(prob, I[a], tol=1e-12).x for a in range(d)]
    st = ds.ga_dual_start(prob, prim, ref["A_up"])
    G = sp.proj_J(prob.N, prob.Y)
    zero = [np.zeros_like(s) for s in st]
    e_start = ga.energy_matrix(prob.Btil, st, list(I))
    e_zero = ga.energy_matrix(prob.Btil, zero, list(I))
    for b in range(d):
        assert np.abs(sp.apply_blockdiag(G, st[b]) - st[b]).max() <= 1e-12 * (np.abs(st[b]).max() + 1.0)
        gap_s = e_start[b, b] - ref["B_up"][b, b]
        gap_z = e_zero[b, b] - ref["B_up"][b, b]
        assert gap_s >= -1e-12 * ref["B_up"][b, b]
        # not exact for the Ga pair (measured 0.19 and 0.12 of the zero start's excess here)
        assert gap_s <= 0.25 * gap_z, (gap_s, gap_z)
        r = ga.solve(prob, I[b], dual=True, tol=1e-12, x0=st[b])
        assert np.abs(ga.energy_matrix(prob.Btil, [r.x], [I[b]])[0, 0] - ref["B_up"][b, b]) <= \
            1e-10 * ref["B_up"][b, b]
