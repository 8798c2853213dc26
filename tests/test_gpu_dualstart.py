"""GPU: the dual start from the primal minimisers (hom_dual_start).

Proposition FD_odd_problem (ii), eq. FD_superposition_odd_A, and the remark on
avoiding the dual solution: J + j0 = A sum_a E_a (e_a + x^(a)) with
E = Abar^-1 J, projected onto J_N.  Against the oracle's start element by
element (the same primal fields in), and what it saves: in GaNi mode on odd
grids the start from converged primal minimisers is the dual minimiser (no CG
iteration left), with the exact scheme it is an admissible start closer to the
dual minimiser than zero."""
import numpy as np
import pytest

import homgen
from oracle import dualstart as ds, galerkin as ga

pytestmark = pytest.mark.gpu


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def _aniso_rects(seed=3):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


CASES = [
    ("pix_N13", lambda: homgen.pixel_cell(seed=21, P=25, values=(1.0, 20.0)), (13, 13)),
    ("aniso_N13x41", _aniso_rects, (13, 41)),
    ("sph3d_N5x13x5", lambda: homgen.sphere_cell(seed=22, n=3, anisotropic=True), (5, 13, 5)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make,N", CASES, ids=[c[0] for c in CASES])
def test_dual_start_matches_oracle(name, make, N, precision):
    H = _H()
    import torch
    from layout import field_from_spectrum, spectrum_from_field
    cell = make()
    d = cell.d
    Y = tuple(cell.Y)
    prob = ga.make_problem(cell, N)
    I = np.eye(d)
    prim = [ga.solve(prob, I[a], tol=1e-12).x for a in range(d)]
    Abar = ga.energy_matrix(prob.Atil, prim, list(I))
    ref = ds.ga_dual_start(prob, prim, Abar)
    pb = H.problem_from_cell(cell, N, precision=precision)
    xp = [torch.tensor(field_from_spectrum(x, d, N, Y, False), dtype=torch.complex128, device="cuda") for x in prim]
    out = pb.dual_start(xp, Abar)
    # mixed: one FP32 operator application (three transform axes in 3D)
    tol = 1e-11 if precision == "fp64" else 5e-6
    for b in range(d):
        got = spectrum_from_field(out[b].cpu().numpy(), d, N, Y, True)
        err = np.abs(got - ref[b]).max() / np.abs(ref[b]).max()
        print(f"[dual-start] {name} {precision} load {b}: {err:.1e}", flush=True)
        assert err <= tol


def _paper_square(rho):
    c = homgen.Inclusions(d=2, Y=np.array([2.0, 2.0]), A0=np.eye(2))
    c.add("rect", [0.0, 0.0], [1.2, 1.2], (1.0 + rho) * np.eye(2))
    return c


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gani_dual_start_is_the_dual_minimiser(precision):
    """GaNi, odd grid N = 45 (the paper's cell, contrast 10): from the converged
    primal minimisers and A_{H,N}, the dual CG has nothing left to do."""
    H = _H()
    cell = _paper_square(10.0)
    pb = H.problem_from_cell(cell, (45, 45), precision=precision, M=(125, 125))
    pb.set_gani_from_cell(cell)
    tol = 1e-10 if precision == "fp64" else 1e-8
    r = pb.solve_bounds(tol=tol)
    AHN, BHN = pb.gani_matrices(r["fields_primal"], r["fields_dual"])
    # one side only: the same A_{H,N}, B_{H,N} NaN
    A1, B1 = pb.gani_matrices(r["fields_primal"])
    assert np.array_equal(A1, AHN) and np.isnan(B1).all()
    x0 = pb.dual_start(r["fields_primal"], AHN)
    xs, info = pb.solve(True, x0=x0, tol=10 * tol)
    its0 = [i["iters"] for i in r["info_dual"]]
    its = [i["iters"] for i in info]
    print(f"[dual-start] GaNi {precision}: dual iterations from zero {its0}, from the start {its}", flush=True)
    assert max(its) <= 2
    b = pb.bounds(dual=xs)
    assert np.abs(b["A_low"] - r["A_low"]).max() <= (1e-9 if precision == "fp64" else 1e-5) * np.abs(r["A_low"]).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ga_dual_start_is_admissible_and_saves_iterations(precision):
    H = _H()
    for seed in (6_000_001, 6_000_002):
        cell = homgen.random_squares_cell(seed, logrho=(2.0, 3.0))[0]
        pb = H.problem_from_cell(cell, (63, 63), precision=precision)
        tol = 1e-10 if precision == "fp64" else 1e-6
        r = pb.solve_bounds(tol=tol)
        x0 = pb.dual_start(r["fields_primal"], r["A_up"])
        start = pb.bounds(dual=x0)
        zero = pb.bounds(dual=[pb.new_field(True) for _ in range(2)])
        xs, info = pb.solve(True, x0=x0, tol=tol)
        b = pb.bounds(dual=xs)
        its0 = [i["iters"] for i in r["info_dual"]]
        its = [i["iters"] for i in info]
        ex_s = np.diag(start["B_up"]) - np.diag(r["B_up"])
        ex_z = np.diag(zero["B_up"]) - np.diag(r["B_up"])
        print(f"[dual-start] Ga {precision} cell {seed}: dual energy excess of the start {ex_s / ex_z} of the zero "
              f"start's; iterations {its0} -> {its}", flush=True)
        # an admissible start: its energy bounds the converged one from above, and improves on zero
        assert (ex_s >= -1e-9 * np.diag(r["B_up"])).all() and (ex_s < ex_z).all()
        assert np.abs(b["A_low"] - r["A_low"]).max() <= 1e-6 * np.abs(r["A_low"]).max()
        # under the guaranteed energy rule, which stops on the energy the start improves
        a_min, a_max = H.cell_eig_range(cell)
        pb.set_stop("guaranteed", 1e-7, a_min=a_min, a_max=a_max)
        _, iz = pb.solve(True, tol=1e-14, maxit=3000, allow_not_converged=True)
        _, i1 = pb.solve(True, x0=x0, tol=1e-14, maxit=3000, allow_not_converged=True)
        pb.set_stop("residual")
        print(f"[dual-start] Ga {precision} cell {seed}, guaranteed rule 1e-7: iterations "
              f"{[i['iters'] for i in iz]} -> {[i['iters'] for i in i1]}", flush=True)
