"""GPU: tile shapes of the specialised FP32 passes.

Every shape computes the same method.  A column-pass shape changes only which
threads transform which points; each instantiation may still fuse multiplies
and adds differently, so results agree to FP32 rounding of the fields, which
enters the FP64 bounds squared (1e-12 relative).  A row-pass shape changes the
blocking of the CG reductions (1e-10 relative on the bounds, iteration counts
within one).  The tuner reports a timed choice, and pinned shapes are
validated."""
import numpy as np
import pytest

import homgen

pytestmark = pytest.mark.gpu

# doubled-grid length -> (row shapes (pairs, threads), column shapes (points, half exchange, all packs))
SHAPES = {
    25: ([(25, 0), (12, 0), (6, 0), (12, 256), (6, 256)],
         [(51, 0, 0), (25, 0, 0), (51, 1, 0), (25, 1, 0), (25, 0, 1), (25, 1, 1)]),
    81: ([(14, 0), (7, 0), (4, 0), (2, 0), (7, 256), (4, 256), (2, 256)],
         [(28, 0, 0), (14, 0, 0), (28, 1, 0), (14, 1, 0), (14, 0, 1), (14, 1, 1)]),
    125: ([(4, 0), (2, 0), (1, 0), (2, 256), (1, 256)],
          [(10, 0, 0), (5, 0, 0), (10, 1, 0), (5, 1, 0), (5, 0, 1), (5, 1, 1)]),
    625: ([(2, 0), (1, 0), (4, 0), (2, 256), (1, 256)],
          [(8, 0, 0), (10, 1, 0), (20, 1, 0), (5, 1, 0), (10, 1, 1), (5, 1, 1)]),
}


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def relerr(X, R):
    return float(np.abs(np.asarray(X) - np.asarray(R)).max() / np.linalg.norm(np.asarray(R), 2))


def _batch(H, N, seeds):
    import torch
    st = torch.cuda.Stream()
    cells = [homgen.pixel_cell(seed=s, P=25, values=(1.0, 30.0 + 20 * i)) for i, s in enumerate(seeds)]
    probs = [H.problem_from_cell(c, N, precision="mixed", max_loads=2, stream=st) for c in cells]
    return probs, H.Batch(probs)


def _pin(b, **shape):
    for dual in (False, True):
        b.set_tiles(dual, 2, **shape)


def _iters(out):
    return [[i["iters"] for i in r["info_primal"] + r["info_dual"]] for r in out]


@pytest.mark.parametrize("N", [13, 41, 63, 313], ids=["M25", "M81", "M125", "M625"])
def test_every_tile_shape_gives_the_same_bounds(N):
    H = _H()
    M = 2 * N - 1
    rows, cols = SHAPES[M]
    probs, b = _batch(H, (N, N), [900 + N, 901 + N])
    _pin(b)
    ref = b.solve_bounds(tol=1e-8)
    print(f"[tiles] M={M} default iterations {_iters(ref)}", flush=True)
    for tp, hx, al in cols:
        _pin(b, apply_points=tp, apply_half_exchange=hx, apply_all_packs=al)
        out = b.solve_bounds(tol=1e-8)
        for r, o in zip(ref, out):
            assert relerr(o["A_up"], r["A_up"]) <= 1e-12 and relerr(o["A_low"], r["A_low"]) <= 1e-12, (tp, hx, al)
        for a, c in zip(_iters(out), _iters(ref)):
            assert max(abs(x - y) for x, y in zip(a, c)) <= 1
    for G, thr in rows:
        _pin(b, row_pairs=G, row_threads=thr)
        out = b.solve_bounds(tol=1e-8)
        for r, o in zip(ref, out):
            assert relerr(o["A_up"], r["A_up"]) <= 1e-10 and relerr(o["A_low"], r["A_low"]) <= 1e-10, (G, thr)
        for a, c in zip(_iters(out), _iters(ref)):
            assert max(abs(x - y) for x, y in zip(a, c)) <= 1
    with pytest.raises(H.HomError):
        b.set_tiles(False, 2, row_pairs=3)
    with pytest.raises(H.HomError):
        b.set_tiles(False, 2, apply_points=7)
    with pytest.raises(H.HomError):
        b.set_tiles(False, 2, row_threads=96)
    with pytest.raises(H.HomError):
        b.set_tiles(False, 2, apply_points=cols[0][0], apply_half_exchange=cols[0][1], apply_all_packs=1)


def test_tuner_reports_a_timed_choice_and_batch_matches_single():
    H = _H()
    # N = 41 with one load: a geometry no other test of this file tunes first
    probs, b = _batch(H, (41, 41), [1201, 1202, 1203])
    t = b.tuning(False, 1)
    print(f"[tiles] tuned {t}", flush=True)
    assert t["candidates"] >= 3 and t["row_ms"] > 0 and t["apply_ms"] > 0
    assert t["row_pairs"] in (14, 7, 4, 2)
    assert (t["apply_points"], t["apply_half_exchange"], t["apply_all_packs"]) in SHAPES[81][1]
    # every later solve of the geometry, batched or single, uses the same choice
    E = np.array([[1.0, 0.0]])
    xb, ib = b.solve(False, E=E, tol=1e-8)
    for i, p in enumerate(probs):
        assert p.tuning(False, 1)["row_pairs"] == t["row_pairs"]
        xs, is_ = p.solve(False, E=E, tol=1e-8)
        assert bool((xs[0] == xb[i][0]).all()) and is_[0]["iters"] == ib[i][0]["iters"]


def test_fp64_problems_reject_pinned_tiles():
    H = _H()
    cell = homgen.square_inclusion_cell()
    pb = H.problem_from_cell(cell, (13, 13), precision="fp64")
    with pytest.raises(H.HomError):
        pb.set_tiles(False, 2, row_pairs=25)
    assert pb.tuning(False, 2)["candidates"] == 0


def test_tuner_cache_persists_choices(tmp_path):
    """A tuned choice written to disk and read back after the process cache was
    emptied is the one later batches of the geometry use (its recorded timings
    come from the file, not from a new timing run), and gives the same bounds."""
    H = _H()
    from paper_1404_3614_amd import api
    probs, b = _batch(H, 41, [101, 102])
    t0 = b.tuning(False, 2)
    ref = b.solve_bounds(tol=1e-8)
    path = tmp_path / "tune.jsonl"
    api.tune_cache_save(path)
    api.tune_cache_clear()
    assert api.tune_cache_load(path) >= 1
    probs2, b2 = _batch(H, 41, [101, 102])
    t1 = b2.tuning(False, 2)
    for k in ("row_pairs", "row_threads", "apply_points", "apply_half_exchange", "apply_all_packs", "candidates"):
        assert t1[k] == t0[k], k
    for k in ("row_ms", "apply_ms"):       # written with 9 significant digits
        assert abs(t1[k] - t0[k]) <= 1e-8 * abs(t0[k]), k
    out = b2.solve_bounds(tol=1e-8)
    for x, y in zip(out, ref):
        assert np.array_equal(x["A_up"], y["A_up"]) and np.array_equal(x["A_low"], y["A_low"])
