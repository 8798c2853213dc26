"""GPU parity at the sizes the measurements run: the N = 63 class (doubled grid
125, the specialised FP32 kernels of the learned-start and mixed-batch
workloads) and a sample of the mixed batch (one cell of every size class at
the highest contrast the batch draws, up to 1e3), against the FP64 oracle.

Reference values: the oracle run live where it finishes in seconds (N <= 63),
else the golden entries "C4s_*" of tests/golden/reference_bounds.json, written
by `python -m oracle.make_golden` (oracle only, CG to 1e-11).

Tolerances (relative bound error, max_ab |X - X_ref|_ab / ||X_ref||_2):
  * FP64, CG to 1e-10: 1e-9 (the bound error is quadratic in the field error,
    Lemma estimates: ~ contrast x 1e-20, far below rounding);
  * mixed, CG to 1e-6 (the workloads' tolerance): 1e-6, the required accuracy
    (FP32 transforms perturb the field, which enters the bound squared; the
    bound quadrature is FP64);
  * operator, element by element: 1e-12 (FP64) and 2e-6 (mixed) of the
    result's largest entry, as for the smaller grids.
"""
import json
import os

import numpy as np
import pytest

import homgen
from oracle import galerkin as ga, make_golden, spectral as sp

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reference_bounds.json")
SAMPLE = make_golden.c4_sample()        # {name: (batch index, N, cell, rho)}


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def relerr(X, R):
    return float(np.abs(np.asarray(X) - np.asarray(R)).max() / np.linalg.norm(np.asarray(R), 2))


def golden(name):
    with open(GOLDEN) as f:
        g = json.load(f)[name]
    return {k: np.array(g[k]) for k in ("A_up", "A_low")}, g


def check(res, ref, tol, what):
    for key in ("A_up", "A_low"):
        e = relerr(res[key], ref[key])
        print(f"[configs] {what} {key} err {e:.2e}", flush=True)
        assert e <= tol, (what, key, e)
    ev = np.linalg.eigvalsh(0.5 * (res["A_up"] - res["A_low"]) + 0.5 * (res["A_up"] - res["A_low"]).T)
    assert ev.min() >= -1e-10 * np.linalg.norm(res["A_up"], 2), "lower bound above the upper bound"


def n63_cells():
    i, N, cell, rho = SAMPLE["C4s_2d_N63"]
    assert N == 63 and rho > 900
    others = [homgen.random_squares_cell(6000000 + s, logrho=(2.0, 3.0))[0] for s in range(3)]
    return cell, others


def test_golden_sample_is_the_batch():
    """The golden entries are the cells the sample picks today (same seeds, same
    geometry generator): index, grid and contrast agree."""
    for name, (i, N, cell, rho) in SAMPLE.items():
        ref, g = golden(name)
        assert g["batch_index"] == i and g["N"][0] == N and abs(g["rho"] - rho) <= 1e-12 * rho, name


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_operator_n63_matches_oracle(prec, dual):
    """One operator application on Z_63 (doubled grid 125: the register
    four-step 125 = 25 x 5 kernels in mixed precision) element by element."""
    import torch
    from layout import field_from_spectrum
    H = _H()
    cell, _ = n63_cells()
    N = (63, 63)
    pb = H.problem_from_cell(cell, N, precision=prec)
    op = ga.make_problem(cell, N)
    rng = np.random.default_rng(63)
    u = rng.standard_normal((2,) + N)
    G = sp.proj_J(N, np.array(cell.Y)) if dual else sp.proj_E(N, np.array(cell.Y))
    xh = sp.apply_blockdiag(G, sp.dft_nd(u, 2))
    c = field_from_spectrum(xh, 2, N, cell.Y, dual)
    y = pb.apply(torch.tensor(c, dtype=torch.complex128, device="cuda"), dual).cpu().numpy()
    yo = field_from_spectrum(sp.apply_blockdiag(G, ga.ga_apply(op.Btil if dual else op.Atil, xh, N)),
                             2, N, cell.Y, dual)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"[configs] operator N=63 {prec} dual={dual}: {err:.2e}", flush=True)
    assert err <= (1e-12 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-9), ("mixed", 1e-6, 1e-6)], ids=["fp64", "mixed"])
def test_single_n63_high_contrast_matches_oracle(prec, tol, bar):
    H = _H()
    cell, _ = n63_cells()
    ref, _ = golden("C4s_2d_N63")
    res = H.problem_from_cell(cell, 63, precision=prec).solve_bounds(tol=tol)
    check(res, ref, bar, f"single N=63 {prec}")


@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-9), ("mixed", 1e-6, 1e-6)], ids=["fp64", "mixed"])
def test_batched_n63_matches_oracle(prec, tol, bar):
    """A lockstep batch of four N = 63 cells (contrast 1e2 .. 1e3): the golden
    cell and one other against the oracle, every cell against its own single
    solve (same kernels: equal to rounding of the reduction order)."""
    import torch
    H = _H()
    cell, others = n63_cells()
    cells = [cell] + others
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, 63, precision=prec, stream=st) for c in cells]
    out = H.Batch(probs).solve_bounds(tol=tol)
    ref, _ = golden("C4s_2d_N63")
    check(out[0], ref, bar, f"batched N=63 {prec} golden cell")
    ref1 = ga.bounds(ga.make_problem(others[0], (63, 63)), tol=1e-11)
    check(out[1], ref1, bar, f"batched N=63 {prec} cell 1")
    for i, c in enumerate(cells):
        single = H.problem_from_cell(c, 63, precision=prec).solve_bounds(tol=tol)
        for key in ("A_up", "A_low"):
            assert relerr(out[i][key], single[key]) <= 1e-9


# column-pass shapes (points per block, half exchange, all packs in one block) of the doubled grid 125
SHAPES_125 = [(10, 0, 0), (5, 0, 0), (10, 1, 0), (5, 1, 0), (5, 0, 1), (5, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES_125, ids=[f"p{a}h{b}a{c}" for a, b, c in SHAPES_125])
def test_n63_every_tile_shape_matches_oracle(shape):
    """Each candidate column-pass shape the tuner may pick for the doubled grid
    125, pinned, gives the oracle's bounds at the mixed tolerance."""
    import torch
    H = _H()
    cell, others = n63_cells()
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, 63, precision="mixed", stream=st) for c in (cell, others[1])]
    b = H.Batch(probs)
    for dual in (False, True):
        b.set_tiles(dual, 2, apply_points=shape[0], apply_half_exchange=shape[1], apply_all_packs=shape[2])
    out = b.solve_bounds(tol=1e-6)
    ref, _ = golden("C4s_2d_N63")
    check(out[0], ref, 1e-6, f"N=63 shape {shape}")


def sample_batch(extra_per_class=3):
    """The golden cell of every size class plus the first `extra_per_class`
    other cells of that class in the default mixed batch."""
    specs = homgen.batch_specs()
    picked = {i: name for name, (i, N, cell, rho) in SAMPLE.items()}
    count = {}
    chosen = []
    for i, (N, cell, rho) in enumerate(specs):
        key = (cell.d, N)
        if i in picked:
            chosen.append((i, N, cell, picked[i]))
        elif count.get(key, 0) < extra_per_class:
            count[key] = count.get(key, 0) + 1
            chosen.append((i, N, cell, None))
    return chosen


@pytest.mark.parametrize("prec,tol,bar", [("mixed", 1e-6, 1e-6), ("fp64", 1e-10, 1e-9)], ids=["mixed", "fp64"])
def test_mixed_batch_sample_matches_oracle(prec, tol, bar):
    """A sample of the mixed batch (20 cells: every 2D class N = 13, 41, 63, 313
    and the 3D class N = 41, each with its highest-contrast cell) through the
    same MixedSolver path the batch measurement runs, classes concurrent on
    their own streams; the golden cells against the oracle."""
    H = _H()
    from paper_1404_3614_amd.mixed import MixedSolver
    chosen = sample_batch()
    print(f"[configs] sample of {len(chosen)} cells: "
          f"{sorted(set((c.d, N) for _, N, c, _ in chosen))}", flush=True)
    ms = MixedSolver(precision=prec)
    groups = ms.prepare([(N, c) for _, N, c, _ in chosen])
    res = ms.solve(groups, len(chosen), tol=tol)
    seen = 0
    for k, (i, N, cell, name) in enumerate(chosen):
        r = res[k]
        ev = np.linalg.eigvalsh(0.5 * (r["A_up"] - r["A_low"]) + 0.5 * (r["A_up"] - r["A_low"]).T)
        assert ev.min() >= -1e-10 * np.linalg.norm(r["A_up"], 2)
        if name is None:
            continue
        ref, _ = golden(name)
        check(r, ref, bar, f"{name} ({prec}, batch cell {i})")
        seen += 1
    assert seen == len(SAMPLE)
