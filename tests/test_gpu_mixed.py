"""GPU: mixed batches of uneven size (cells grouped by size class, each class
one lockstep batch) against the FP64 oracle and against single-cell solves."""
import numpy as np
import pytest

import homgen
from oracle import galerkin as ga

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


def test_mixed_batch_matches_oracle_and_single_solves():
    H = _H()
    from paper_1404_3614_amd.mixed import MixedSolver
    specs = homgen.batch_specs(seed0=4242, n2d=10, n3d=2, Ns2d=(13, 41), N3d=13)
    print(f"[mixed] {len(specs)} cells, N = {[s[0] for s in specs]}", flush=True)
    ms = MixedSolver(precision="mixed")
    groups = ms.prepare([(N, c) for N, c, _ in specs])
    assert sum(len(v) for v in groups.values()) == len(specs)
    res = ms.solve(groups, len(specs), tol=1e-8)
    for i, (N, cell, rho) in enumerate(specs):
        r = res[i]
        assert r["class"]["N"] == tuple([N] * cell.d)
        single = H.problem_from_cell(cell, N, precision="mixed").solve_bounds(tol=1e-8)
        assert relerr(r["A_up"], single["A_up"]) <= 1e-9
        assert relerr(r["A_low"], single["A_low"]) <= 1e-9
        ev = np.linalg.eigvalsh(r["A_up"] - r["A_low"])
        assert ev.min() >= -1e-10 * np.linalg.norm(r["A_up"], 2)
    # oracle on the small 2D cells
    checked = 0
    for i, (N, cell, rho) in enumerate(specs):
        if cell.d == 2 and N == 13 and checked < 3:
            op = ga.make_problem(cell, N)
            ref = ga.bounds(op, tol=1e-10)
            assert relerr(res[i]["A_up"], ref["A_up"]) <= 1e-6
            assert relerr(res[i]["A_low"], ref["A_low"]) <= 1e-6
            checked += 1
    assert checked >= 1
    # a second call with new cells of the same classes re-uses the class batches
    specs2 = homgen.batch_specs(seed0=5151, n2d=10, n3d=2, Ns2d=(13, 41), N3d=13)
    keys_before = set(ms.classes)
    groups2 = ms.prepare([(N, c) for N, c, _ in specs2])
    res2 = ms.solve(groups2, len(specs2), tol=1e-8)
    for i, (N, cell, rho) in enumerate(specs2):
        single = H.problem_from_cell(cell, N, precision="mixed").solve_bounds(tol=1e-8)
        assert relerr(res2[i]["A_up"], single["A_up"]) <= 1e-9
    assert keys_before <= set(ms.classes)
