"""GPU: the gap rule (stop each side once its remaining error is below theta
times a guaranteed lower bound on the converged gap of its bound; primal and
dual side by side in lockstep chunks; Sec. 7.2 Convergence-criteria remark,
eq. approx_homog_with_error) against the oracle's lockstep CG with the same
rule (oracle/stopping.py, solve_pair_gap).

Bars: stopping iterations within one of the oracle's in FP64 (the Gauss-Radau
bound crosses the threshold within rounding), two in mixed precision (the
FP32 operator perturbs the CG scalars at 1e-7); every final bound within
theta D* of the converged one (D* = U* - |E|^4 / V* from the oracle at 1e-11,
plus 2e-7 U* of FP32 rounding in mixed precision), and on the guaranteed
side of it.
"""
import numpy as np
import pytest

import homgen
from oracle import galerkin as ga, stopping as stp

pytestmark = pytest.mark.gpu

CHUNK = 8     # iterations per captured chunk (the library's default)


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def _cells():
    return [homgen.random_squares_cell(7100 + s, logrho=(1.5, 3.0))[0] for s in range(3)]


_CONVERGED = {}


def converged(i, cell, N):
    """Oracle bounds at 1e-11 (cached across the parametrisations)."""
    if (i, N) not in _CONVERGED:
        _CONVERGED[i, N] = ga.bounds(ga.make_problem(cell, N), tol=1e-11)
    return _CONVERGED[i, N]


def _batch(H, cells, N, precision, theta):
    import torch
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, N, precision=precision, stream=st) for c in cells]
    b = H.Batch(probs)
    rng = [H.cell_eig_range(c) for c in cells]
    a_min, a_max = min(r[0] for r in rng), max(r[1] for r in rng)
    b.set_stop("gap", theta, a_min, a_max)
    return b, (a_min, 1.0 / a_max)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("theta", [1e-1, 1e-3])
def test_gap_rule_matches_oracle(precision, theta):
    H = _H()
    N = (41, 41)
    cells = _cells()
    b, mu = _batch(H, cells, N, precision, theta)
    out = b.solve_bounds(tol=1e-14, maxit=4000, allow_not_converged=True)
    slack_it = 1 if precision == "fp64" else 2
    for i, c in enumerate(cells):
        prob = ga.make_problem(c, N)
        conv = converged(i, c, N)
        for a in range(2):
            E = np.eye(2)[a]
            P, D, dlow = stp.solve_pair_gap(prob, E, tol=1e-14, theta=theta, chunk=CHUNK, mu=mu)
            gp, gd = out[i]["info_primal"][a]["iters"], out[i]["info_dual"][a]["iters"]
            print(f"[gap] {precision} theta {theta:g} cell {i} load {a}: gpu {gp}/{gd} oracle {P.i}/{D.i} "
                  f"({P.status}/{D.status})", flush=True)
            assert abs(gp - P.i) <= slack_it and abs(gd - D.i) <= slack_it
            U_star, V_star = conv["A_up"][a, a], conv["B_up"][a, a]
            D_star = U_star - 1.0 / V_star
            U, V = out[i]["A_up"][a, a], out[i]["B_up"][a, a]
            slack = 0.0 if precision == "fp64" else 2e-7 * U_star
            assert U >= U_star * (1 - 1e-12) - slack and 1.0 / V <= 1.0 / V_star * (1 + 1e-12) + slack
            assert U - U_star <= theta * D_star + 1e-12 * U_star + slack
            assert 1.0 / V_star - 1.0 / V <= theta * D_star + 1e-12 * U_star + slack
        # the bounds stay guaranteed as matrices
        n = np.linalg.norm(conv["A_up"], 2)
        assert np.linalg.eigvalsh(out[i]["A_up"] - conv["A_up"]).min() >= -1e-9 * n
        assert np.linalg.eigvalsh(conv["A_low"] - out[i]["A_low"]).min() >= -1e-9 * n


def test_gap_rule_deterministic_across_launch_modes():
    """Graph replay with the two solves concurrent and direct launches one
    chunk at a time (the timing mode) stop at the same iterations with the
    same bounds: each chunk reads the partner's state of the previous one."""
    H = _H()
    cells = _cells()
    b, _ = _batch(H, cells, (41, 41), "mixed", 1e-2)
    g = b.solve_bounds(tol=1e-14, maxit=4000, allow_not_converged=True)
    b.set_timing(True)
    t = b.solve_bounds(tol=1e-14, maxit=4000, allow_not_converged=True)
    b.set_timing(False)
    for x, y in zip(g, t):
        assert [i["iters"] for i in x["info_primal"] + x["info_dual"]] == \
            [i["iters"] for i in y["info_primal"] + y["info_dual"]]
        assert np.array_equal(x["A_up"], y["A_up"]) and np.array_equal(x["A_low"], y["A_low"])


def test_gap_rule_needs_the_pair_solve():
    H = _H()
    cell = _cells()[0]
    pb = H.problem_from_cell(cell, (13, 13), precision="mixed")
    pb.set_stop("gap", 1e-2, 1.0, 1e3)
    with pytest.raises(H.HomError):
        pb.solve(False, tol=1e-8)
    b, _ = _batch(H, [cell], (13, 13), "mixed", 1e-2)
    with pytest.raises(H.HomError):
        b.solve(False, tol=1e-8)
    r = b.solve_bounds(tol=1e-14, maxit=4000, allow_not_converged=True)
    assert np.linalg.eigvalsh(r[0]["A_up"] - r[0]["A_low"]).min() >= 0
