"""GPU: quadrature grids larger than 2N - 1, point values on the N grid, and
the GaNi scheme (Def. GaNi, the paper's Algorithm) against the FP64 oracle.

A quadrature grid M >= 2N - 1 integrates the bilinear forms of Z_N fields
exactly (no product frequency aliases onto Z_N), so the bounds on any such
grid equal those of the oracle's doubled grid.  GaNi solves with the point
values of A on the N grid and N-point transforms; its minimisers still give
guaranteed bounds through the exact quadrature (step (iii))."""
import numpy as np
import pytest

import homgen
from oracle import coefficients as co, galerkin as ga, gani

pytestmark = pytest.mark.gpu


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def relerr(X, R):
    return float(np.abs(np.asarray(X) - np.asarray(R)).max() / np.linalg.norm(np.asarray(R), 2))


def _aniso_rects(seed=21):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


# (name, cell, N, quadrature grid M)
GRIDS = [
    ("square_N13_M27", lambda: homgen.square_inclusion_cell(rho_in=10.0), (13, 13), (27, 27)),
    ("aniso_N15_M45", _aniso_rects, (15, 9), (45, 25)),
    ("pix_N15_M45", lambda: homgen.pixel_cell(seed=7, P=25, values=(1.0, 20.0)), (15, 15), (45, 45)),
    ("sph3d_N5_M15", lambda: homgen.sphere_cell(seed=8, n=3, anisotropic=True), (5, 5, 5), (15, 9, 15)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make,N,M", GRIDS, ids=[g[0] for g in GRIDS])
def test_larger_quadrature_grid_is_exact(name, make, N, M, precision):
    H = _H()
    cell = make()
    pb = H.problem_from_cell(cell, N, precision=precision, M=M)
    assert pb.M == tuple(M)
    r = pb.solve_bounds(tol=1e-10 if precision == "fp64" else 1e-8)
    ref = ga.bounds(ga.make_problem(cell, N), tol=1e-11)
    tol = 1e-9 if precision == "fp64" else 1e-6
    eu, el = relerr(r["A_up"], ref["A_up"]), relerr(r["A_low"], ref["A_low"])
    print(f"[grid] {name} {precision}: A_up {eu:.2e} A_low {el:.2e}", flush=True)
    assert eu <= tol and el <= tol


def test_quadrature_grid_validation():
    H = _H()
    cell = homgen.square_inclusion_cell()
    for M in ((23, 23), (26, 25), (49, 49)):        # below 2N - 1, even, factor 7
        with pytest.raises(H.HomError):
            H.problem_from_cell(cell, (13, 13), M=M)


def _components(full, nc):
    """(d, d, *N) matrices -> [nc] components in the library's order."""
    d = full.shape[0]
    if nc == 1:
        return full[0, 0][None]
    if d == 2:
        return np.stack([full[0, 0], full[1, 1], full[0, 1]])
    return np.stack([full[0, 0], full[1, 1], full[2, 2], full[0, 1], full[0, 2], full[1, 2]])


SAMPLES = [
    ("square", lambda: homgen.square_inclusion_cell(rho_in=10.0), (13, 13)),
    ("aniso", _aniso_rects, (15, 9)),
    ("pix", lambda: homgen.pixel_cell(seed=9, P=25, values=(1.0, 30.0)), (45, 15)),
    ("sph3d", lambda: homgen.sphere_cell(seed=10, n=6, anisotropic=True), (9, 15, 5)),
]


@pytest.mark.parametrize("inverse", [False, True], ids=["A", "Ainv"])
@pytest.mark.parametrize("name,make,N", SAMPLES, ids=[s[0] for s in SAMPLES])
def test_point_values_match_oracle(name, make, N, inverse):
    """The inside/outside decisions are bitwise those of the oracle (same
    arithmetic, same order); the values agree to the rounding of the inverses."""
    H = _H()
    cell = make()
    nc = H.api.cell_ncoef(cell)
    got = H.sample_cell(cell, N, nc, inverse=inverse).cpu().numpy()
    ref = _components(co.point_values(cell, N, inverse=inverse), nc)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def _paper_square(rho):
    """The cell of the paper's experiments: (-1, 1)^2, square |x_a| < 3/5 of (1 + rho) I in I."""
    c = homgen.Inclusions(d=2, Y=np.array([2.0, 2.0]), A0=np.eye(2))
    c.add("rect", [0.0, 0.0], [1.2, 1.2], (1.0 + rho) * np.eye(2))
    return c


GANI = [
    ("square_N15", lambda: homgen.square_inclusion_cell(rho_in=10.0), (15, 15), (45, 45)),
    ("paper_S_rho10_N5", lambda: _paper_square(10.0), (5, 5), (9, 9)),
    ("paper_S_rho1e3_N45", lambda: _paper_square(1e3), (45, 45), (125, 125)),
    ("aniso_N15x9", _aniso_rects, (15, 9), (45, 25)),
    ("pix_N45", lambda: homgen.pixel_cell(seed=11, P=25, values=(1.0, 50.0)), (45, 45), (125, 125)),
    ("sph3d_N9", lambda: homgen.sphere_cell(seed=12, n=4, anisotropic=True), (9, 9, 9), (25, 25, 25)),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,make,N,M", GANI, ids=[g[0] for g in GANI])
def test_gani_matches_oracle(name, make, N, M, precision):
    H = _H()
    cell = make()
    ref = gani.gani_bounds(cell, N, tol=1e-11)
    pb = H.problem_from_cell(cell, N, precision=precision, M=M)
    ga_r = pb.solve_bounds(tol=1e-10 if precision == "fp64" else 1e-8)
    pb.set_gani_from_cell(cell)
    tol_cg = 1e-10 if precision == "fp64" else 1e-8
    r = pb.solve_bounds(tol=tol_cg)
    AHN, BHN = pb.gani_matrices(r["fields_primal"], r["fields_dual"])
    tol = 1e-9 if precision == "fp64" else 1e-6
    errs = dict(A_HN=relerr(AHN, ref["A_HN"]), B_HN=relerr(BHN, ref["B_HN"]), A_up=relerr(r["A_up"], ref["A_up"]),
                A_low=relerr(r["A_low"], ref["A_low"]))
    its = [i["iters"] for i in r["info_primal"] + r["info_dual"]]
    print(f"[gani] {name} {precision}: {', '.join(f'{k} {v:.1e}' for k, v in errs.items())}; iterations {its} "
          f"oracle {ref['iters']}", flush=True)
    # A_{H,N} is the GaNi energy at its own minimiser: second order in the algebraic error
    assert errs["A_HN"] <= tol and errs["B_HN"] <= tol
    # the exact energy of a GaNi minimiser is not minimal in the exact form, so the bounds
    # are first order in its error; with FP32 transforms that error grows like the square
    # root of the coefficient's contrast
    a_min, a_max = H.cell_eig_range(cell)
    tol_b = tol if precision == "fp64" else tol * np.sqrt(a_max / a_min)
    assert errs["A_up"] <= tol_b and errs["A_low"] <= tol_b
    # the CG energy of the GaNi solve is the diagonal of A_{H,N} (the recurrence of the FP32
    # operator carries its rounding, growing with the contrast like the bounds above)
    ep = np.array([i["energy"] for i in r["info_primal"]])
    assert np.abs(ep - np.diag(AHN)).max() <= tol_b * np.linalg.norm(AHN, 2)
    # odd grids: A_{H,N} = B_{H,N}^{-1}; the exact bounds of the GaNi fields enclose those of the Ga fields
    n = np.linalg.norm(AHN, 2)
    assert relerr(AHN, np.linalg.inv(BHN)) <= (1e-8 if precision == "fp64" else 1e-5)
    assert np.linalg.eigvalsh(r["A_up"] - ga_r["A_up"]).min() >= -1e-9 * n
    assert np.linalg.eigvalsh(ga_r["A_low"] - r["A_low"]).min() >= -1e-9 * n
    # back to the exact operator: the same result as before GaNi mode
    pb.clear_gani()
    again = pb.solve_bounds(tol=1e-10 if precision == "fp64" else 1e-8)
    assert relerr(again["A_up"], ga_r["A_up"]) <= 1e-13 and relerr(again["A_low"], ga_r["A_low"]) <= 1e-13


def test_gani_rejects_batches_and_bad_grids():
    H = _H()
    import torch
    st = torch.cuda.Stream()
    cell = homgen.square_inclusion_cell(rho_in=5.0)
    probs = [H.problem_from_cell(cell, (15, 15), precision="mixed", M=(45, 45), stream=st) for _ in range(2)]
    b = H.Batch(probs)
    probs[0].set_gani_from_cell(cell)
    with pytest.raises(H.HomError):
        b.solve(False, tol=1e-8)
    probs[0].clear_gani()
    b.solve(False, tol=1e-8)
    # N = 13 has a factor 13: no N-point transform
    pb = H.problem_from_cell(cell, (13, 13), precision="mixed")
    with pytest.raises(H.HomError):
        pb.set_gani_from_cell(cell)


def test_smoothing_filter_matches_oracle_and_bounds():
    """Sec. 8.3 smoothing: the device filter is bitwise the oracle's; the smoothed
    medium (17 phases) gives bounds equal to the oracle's, closer together than
    the unsmoothed medium's on the same grid (Ga and GaNi)."""
    H = _H()
    for seed, P in ((1, (25, 25)), (2, (15, 45))):
        rng = np.random.default_rng(seed)
        cell = homgen.Pixels(d=2, Y=np.array([1.0, 1.0]), phase=(rng.random(P) < 0.45).astype(np.int64),
                             phase_A=np.stack([np.eye(2), 30.0 * np.eye(2)]))
        sm = H.smooth_pixel_cell(cell)
        assert (sm.phase == co.smooth_characteristic(cell.phase)).all()
        assert np.allclose(sm.phase_A[16], 30.0 * np.eye(2)) and np.allclose(sm.phase_A[0], np.eye(2))
    cell = homgen.pixel_cell(seed=13, P=25, values=(1.0, 30.0))
    sm = H.smooth_pixel_cell(cell)
    ref = ga.bounds(ga.make_problem(sm, (13, 13)), tol=1e-11)
    r = H.problem_from_cell(sm, (13, 13), precision="mixed").solve_bounds(tol=1e-8)
    assert relerr(r["A_up"], ref["A_up"]) <= 1e-6 and relerr(r["A_low"], ref["A_low"]) <= 1e-6
    raw = H.problem_from_cell(cell, (13, 13), precision="mixed").solve_bounds(tol=1e-8)
    gap = lambda b: np.linalg.norm(b["D"], 2) / np.linalg.norm(b["A_mean"], 2)
    print(f"[smooth] relative gap ||D||/||A_mean||: raw {gap(raw):.4f} smoothed {gap(r):.4f}", flush=True)
    assert gap(r) < gap(raw)
    # GaNi on the pixel grid (grid points at the pixel centres)
    g = gani.gani_bounds(sm, (25, 25), tol=1e-11)
    pb = H.problem_from_cell(sm, (25, 25), precision="fp64", M=(75, 75))
    pb.set_gani_from_cell(sm)
    rg = pb.solve_bounds(tol=1e-10)
    AHN, BHN = pb.gani_matrices(rg["fields_primal"], rg["fields_dual"])
    assert relerr(AHN, g["A_HN"]) <= 1e-9 and relerr(rg["A_up"], g["A_up"]) <= 1e-9
