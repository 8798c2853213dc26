"""GPU: the CG energy recurrence and the energy stopping rule.

CG minimises the energy a(E + x, E + x) over its Krylov spaces, and each step
lowers it by alpha gamma (Sec. 7.1).  Started from zero, the energy reported
at exit is therefore the diagonal of the upper bound (primal) and of B_up, the
inverse of the lower bound (dual); the FP64 quadrature of the returned fields
recomputes both.  The energy rule stops on that quantity.  Every iterate gives
guaranteed bounds (Sec. 6), and the energy of the iterates does not increase,
so bounds from an earlier exit enclose the converged ones."""
import numpy as np
import pytest

import homgen

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


def _aniso_rects(seed=32):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


CELLS = {
    "pix2d": (lambda: homgen.pixel_cell(seed=31, P=25, values=(1.0, 50.0)), 41),
    "aniso2d": (_aniso_rects, (13, 41)),
    "sph3d": (lambda: homgen.sphere_cell(seed=33, n=6, anisotropic=True), 13),
}
# precision -> (residual tolerance of the solve, energy vs bound-diagonal tolerance)
PREC = {"fp64": (1e-10, 1e-10), "mixed": (1e-8, 1e-6)}


@pytest.mark.parametrize("precision", list(PREC))
@pytest.mark.parametrize("name", list(CELLS))
def test_recurrence_energy_is_the_bound_diagonal(name, precision):
    H = _H()
    make, N = CELLS[name]
    cell = make()
    pb = H.problem_from_cell(cell, N, precision=precision)
    tol, etol = PREC[precision]
    r = pb.solve_bounds(tol=tol)
    ep = np.array([i["energy"] for i in r["info_primal"]])
    ed = np.array([i["energy"] for i in r["info_dual"]])
    dp = np.abs(ep - np.diag(r["A_up"])).max() / np.linalg.norm(r["A_up"], 2)
    dd = np.abs(ed - np.diag(r["B_up"])).max() / np.linalg.norm(r["B_up"], 2)
    print(f"[energy] {name} {precision}: primal {dp:.2e} dual {dd:.2e}", flush=True)
    assert dp <= etol and dd <= etol
    # from a given start the energy of the start enters too: from the converged field
    # (no iteration) and from half of it
    for scale in (1.0, 0.5):
        x0 = [f * scale for f in r["fields_primal"]]
        xs, info = pb.solve(False, x0=x0, tol=tol)
        b = pb.bounds(primal=xs)
        dw = np.abs(np.array([i["energy"] for i in info]) - np.diag(b["A_up"])).max() / np.linalg.norm(b["A_up"], 2)
        print(f"[energy] {name} {precision}: warm start x {scale}: {dw:.2e}", flush=True)
        assert dw <= etol


def _solve_rule(b_or_pb, rule, etol, tol):
    b_or_pb.set_stop(rule, etol)
    out = b_or_pb.solve_bounds(tol=tol, maxit=2000, allow_not_converged=True)
    b_or_pb.set_stop("residual")
    return out


def _iters(r):
    return [i["iters"] for i in r["info_primal"] + r["info_dual"]]


def _zero_field_energy(pb, dual):
    _, info = pb.solve(dual, tol=1e-30, maxit=0, allow_not_converged=True)
    assert all(i["iters"] == 0 for i in info)
    return np.array([i["energy"] for i in info])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_energy_rule_bounds_enclose_the_converged_ones(precision):
    H = _H()
    cell = homgen.pixel_cell(seed=41, P=25, values=(1.0, 100.0))
    pb = H.problem_from_cell(cell, 41, precision=precision)
    ref = pb.solve_bounds(tol=1e-10 if precision == "fp64" else 1e-8)
    # zero-field energies: E^T <A> E and J^T <A^-1> J on the unit loads, the Voigt and
    # Reuss bounds that any iterate improves on
    e0p, e0d = _zero_field_energy(pb, False), _zero_field_energy(pb, True)
    assert (e0p >= np.diag(ref["A_up"]) * (1 - 1e-12)).all() and (e0d >= np.diag(ref["B_up"]) * (1 - 1e-12)).all()
    n = np.linalg.norm(ref["A_up"], 2)
    for etol in (1e-3, 1e-5, 1e-8):
        # the residual rule with a tolerance no solve reaches first: the energy rule decides
        r = _solve_rule(pb, "energy", etol, 1e-14)
        assert all(i["status"] == 0 for i in r["info_primal"] + r["info_dual"]), etol
        ex_p = (np.diag(r["A_up"]) - np.diag(ref["A_up"])) / np.diag(ref["A_up"])
        ex_d = (np.diag(r["B_up"]) - np.diag(ref["B_up"])) / np.diag(ref["B_up"])
        print(f"[energy] {precision} etol {etol:g}: iterations {_iters(r)} vs residual rule {_iters(ref)}; "
              f"relative excess over the converged energy: primal {ex_p.max():.2e} dual {ex_d.max():.2e}",
              flush=True)
        # bounds stay ordered and enclose the converged ones
        assert np.linalg.eigvalsh(r["A_up"] - r["A_low"]).min() >= -1e-9 * n
        assert np.linalg.eigvalsh(r["A_up"] - ref["A_up"]).min() >= -1e-7 * n
        assert np.linalg.eigvalsh(ref["A_low"] - r["A_low"]).min() >= -1e-7 * n
        # each energy within the requested fraction of its converged value
        assert ex_p.max() <= etol + 1e-7 and ex_d.max() <= etol + 1e-7
        if etol <= 1e-8:
            assert relerr(r["A_up"], ref["A_up"]) <= 1e-6 and relerr(r["A_low"], ref["A_low"]) <= 1e-6


def test_energy_rule_batch_equals_single_and_validation():
    H = _H()
    import torch
    st = torch.cuda.Stream()
    cells = [homgen.pixel_cell(seed=s, P=25, values=(1.0, 20.0 + 30 * i)) for i, s in enumerate((51, 52, 53))]
    probs = [H.problem_from_cell(c, 41, precision="mixed", max_loads=2, stream=st) for c in cells]
    b = H.Batch(probs)
    b.set_stop("energy", 1e-6)
    out = b.solve_bounds(tol=1e-12, maxit=2000, allow_not_converged=True)
    for p, o in zip(probs, out):
        p.set_stop("energy", 1e-6)
        s = p.solve_bounds(tol=1e-12, maxit=2000, allow_not_converged=True)
        assert _iters(s) == _iters(o)
        assert relerr(s["A_up"], o["A_up"]) <= 1e-12 and relerr(s["A_low"], o["A_low"]) <= 1e-12
    from paper_1404_3614_amd import _lib as L
    for bad in ((4, 1e-6, 0, 0), (1, 0.0, 0, 0), (1, 1.5, 0, 0), (1, float("nan"), 0, 0), (2, 1e-6, -1.0, 0),
                (2, 1e-6, 2.0, 1.0), (2, 1e-6, float("inf"), 0)):
        with pytest.raises(H.HomError):
            L.check(L.load().hom_batch_set_stop(b.h, *bad), "hom_batch_set_stop")
    with pytest.raises(KeyError):
        probs[0].set_stop("bogus")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_guaranteed_rule_bounds_within_etol(precision):
    H = _H()
    cell = homgen.pixel_cell(seed=61, P=25, values=(1.0, 100.0))
    a_min, a_max = H.cell_eig_range(cell)
    assert (a_min, a_max) == (1.0, 100.0)
    pb = H.problem_from_cell(cell, 41, precision=precision)
    ref = pb.solve_bounds(tol=1e-10 if precision == "fp64" else 1e-8)
    slack = 1e-12 if precision == "fp64" else 2e-7     # FP32 operator rounding
    prev = None
    for etol in (1e-3, 1e-5, 1e-7, 1e-9):
        r = _solve_rule_ab(pb, etol, a_min, a_max)
        its = _iters(r)
        assert all(i["status"] == 0 for i in r["info_primal"] + r["info_dual"]), etol
        ex_p = (np.diag(r["A_up"]) - np.diag(ref["A_up"])) / np.diag(ref["A_up"])
        ex_d = (np.diag(r["B_up"]) - np.diag(ref["B_up"])) / np.diag(ref["B_up"])
        print(f"[guaranteed] {precision} etol {etol:g}: iterations {its} vs residual rule {_iters(ref)}; "
              f"relative excess primal {ex_p.max():.2e} dual {ex_d.max():.2e}", flush=True)
        assert ex_p.max() <= etol + slack and ex_d.max() <= etol + slack
        assert ex_p.min() >= -slack and ex_d.min() >= -slack
        if prev is not None:
            assert all(a >= b for a, b in zip(its, prev))
        prev = its


def _solve_rule_ab(pb, etol, a_min, a_max, tol=1e-14):
    pb.set_stop("guaranteed", etol, a_min=a_min, a_max=a_max)
    out = pb.solve_bounds(tol=tol, maxit=3000, allow_not_converged=True)
    pb.set_stop("residual")
    return out


@pytest.mark.parametrize("given", [True, False], ids=["phase_range", "grid_minimum"])
def test_guaranteed_rule_iterations_match_oracle(given):
    """FP64 path against the oracle's CG with the same rule: the same stopping
    iteration (one apart at most, where the bound crosses etol within rounding)."""
    H = _H()
    from oracle import galerkin as ga, stopping as stp
    # low contrast, so that the doubled-grid minimum is a positive bound as well
    cell = homgen.square_inclusion_cell(rho_in=3.0)
    N = (13, 13)
    prob = ga.make_problem(cell, N)
    a_min, a_max = H.cell_eig_range(cell)
    pb = H.problem_from_cell(cell, N, precision="fp64")
    etol = 1e-9
    out = _solve_rule_ab(pb, etol, a_min if given else 0.0, a_max if given else 0.0)
    for dual in (False, True):
        mu = (1.0 / a_max if dual else a_min) if given else stp.spectrum_lower_bound(prob.Btil if dual else prob.Atil)
        assert mu > 0
        info = out["info_dual" if dual else "info_primal"]
        for a in range(2):
            ref = stp.solve(prob, np.eye(2)[a], dual=dual, tol=1e-14, rule="guaranteed", etol=etol, mu=mu)
            assert ref.status == "energy"
            print(f"[guaranteed] oracle {ref.iters} gpu {info[a]['iters']} (dual={dual}, load {a})", flush=True)
            assert abs(info[a]["iters"] - ref.iters) <= 1
            assert abs(info[a]["energy"] - ref.energy[min(info[a]["iters"], len(ref.energy) - 1)]) <= \
                1e-9 * ref.energy[-1] or info[a]["iters"] > ref.iters
