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


@pytest.mark.parametrize("chunks", [1, 3])
@pytest.mark.parametrize("stop", ["residual", "gap"])
def test_group_graph_equals_per_class_solves(stop, chunks, monkeypatch):
    """All classes from one captured graph (hom_group_solve_pair) against each
    class solved by its own pair solve (host thread per class): the same
    kernels in the same order per cell, so the same iterations and bounds; and
    against the group's direct (timing) mode, which advances the solves one
    chunk each in turn.  chunks: chunks of iterations per graph launch (with
    the gap rule, partner edges between the chunks inside the graph)."""
    if stop == "gap" and chunks > 1:
        pytest.skip("a multi-chunk group graph with in-graph partner edges (cross-stream event waits "
                    "inside the capture) ended the process with a host segmentation fault whose cause "
                    "was not found; under the gap rule the group now captures one chunk per launch")
    _H()
    monkeypatch.setenv("HOM_GROUP_CHUNKS", str(chunks))
    from paper_1404_3614_amd.mixed import MixedSolver
    specs = homgen.batch_specs(seed0=777, n2d=9, n3d=3, Ns2d=(13, 41, 63), N3d=13)
    cells = [(N, c) for N, c, _ in specs]
    kw = dict(precision="mixed", stop=stop, etol=1e-2 if stop == "gap" else None, a_min=1.0, a_max=1e3)
    tol = 1e-8 if stop == "residual" else 1e-14
    out = {}
    for mode in ("graph", "streams", "threads"):
        ms = MixedSolver(mode=mode, **kw)
        groups = ms.prepare(cells)
        out[mode] = ms.solve(groups, len(cells), tol=tol, maxit=3000)
        if mode == "graph":
            again = ms.solve(groups, len(cells), tol=tol, maxit=3000)       # the cached graph
            res_t, _ = ms.solve_timed(groups, len(cells), tol=tol, maxit=3000)
            for a, b, c in zip(out[mode], again, res_t):
                for key in ("A_up", "A_low"):
                    assert np.array_equal(a[key], b[key])
                    assert relerr(a[key], c[key]) <= 1e-13
    its = lambda r: [x["iters"] for x in r["info_primal"] + r["info_dual"]]
    for other in ("streams", "threads"):
        for i, (a, b) in enumerate(zip(out["graph"], out[other])):
            assert its(a) == its(b), (other, i, its(a), its(b))
            for key in ("A_up", "A_low"):
                assert relerr(a[key], b[key]) <= 1e-13, (other, i, key)
