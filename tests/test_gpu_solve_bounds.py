"""hom_batch_solve_bounds: primal and dual solves of the unit loads and their
guaranteed bounds in one call, each side's FP64 bound passes started as soon
as that side has stopped (beside the other side's remaining iterations).

The same kernels run on the same data as hom_batch_solve_pair followed by
hom_batch_bounds, only their order across the two streams changes, so
iterations, fields and bounds must be equal to the bit; one 2D batch is also
checked against the FP64 oracle (Def. upper_lower_bounds: the bounds of the
returned fields, CG to 1e-11 in the oracle, relative bound error within the
mixed-precision tolerance 1e-6 of the CG)."""
import numpy as np
import pytest

import homgen
from oracle import galerkin as ga

pytestmark = pytest.mark.gpu

KEYS = ("A_up", "B_up", "A_low", "A_mean", "D")


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def relerr(X, R):
    return np.abs(np.asarray(X) - np.asarray(R)).max() / np.linalg.norm(np.asarray(R), 2)


def _separate(batch, tol):
    fp, ip, fd, idl = batch.solve_pair(tol=tol, maxit=3000, allow_not_converged=True)
    out = batch.bounds(fp, fd)
    return out, ip, idl, [[t.cpu() for t in f] for f in fp], [[t.cpu() for t in f] for f in fd]


def _fused(batch, tol):
    out = batch.solve_bounds(tol=tol, maxit=3000, allow_not_converged=True)
    d = batch.d
    fp = [[t.cpu() for t in f] for f in batch._fields(False, d)]
    fd = [[t.cpu() for t in f] for f in batch._fields(True, d)]
    return out, [o["info_primal"] for o in out], [o["info_dual"] for o in out], fp, fd


def _same(a, b):
    import torch
    oa, ipa, ida, fpa, fda = a
    ob, ipb, idb, fpb, fdb = b
    for ra, rb in zip(oa, ob):
        for k in KEYS:
            assert np.array_equal(ra[k], rb[k]), k
    for xa, xb in ((ipa, ipb), (ida, idb)):
        for la, lb in zip(xa, xb):
            assert [i["iters"] for i in la] == [i["iters"] for i in lb]
            assert [i["rel_res_true"] for i in la] == [i["rel_res_true"] for i in lb]
            assert [i["energy"] for i in la] == [i["energy"] for i in lb]
    for xa, xb in ((fpa, fpb), (fda, fdb)):
        for la, lb in zip(xa, xb):
            for u, v in zip(la, lb):
                assert torch.equal(u, v)


def _batch(H, cells, N, **kw):
    import torch
    st = torch.cuda.Stream()
    return H.Batch([H.problem_from_cell(c, N, stream=st, **kw) for c in cells])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_2d_fused_equals_separate_and_oracle(prec):
    """Four N = 41 square-inclusion cells (contrast 10 .. 1e3, so the two sides stop at
    different iterations): fused = separate to the bit; cell 0 against the
    oracle."""
    H = _H()
    cells = [homgen.square_inclusion_cell(2, side=0.3 + 0.1 * i, rho_in=10.0 ** (1 + 2 * i / 3)) for i in range(4)]
    batch = _batch(H, cells, 41, precision=prec)
    a = _separate(batch, 1e-6)
    b = _fused(batch, 1e-6)
    its = [(max(i["iters"] for i in p), max(i["iters"] for i in d)) for p, d in zip(b[1], b[2])]
    print(f"[solve_bounds] 2D {prec} iterations (primal, dual) per cell {its}", flush=True)
    _same(a, b)
    ref = ga.bounds(ga.make_problem(cells[0], (41, 41)), tol=1e-11)
    for k in ("A_up", "A_low"):
        assert relerr(b[0][0][k], ref[k]) <= 1e-6, k


def test_3d_plane_geometry_fused_equals_separate():
    """Three N = 41 sphere cells (the plane-pass geometry of the 3D workload)."""
    H = _H()
    cells = [homgen.sphere_cell(seed=80 + i, n=6 + 6 * i, anisotropic=False, rho=10.0 ** (1 + i)) for i in range(3)]
    batch = _batch(H, cells, (41, 41, 41), precision="mixed")
    a = _separate(batch, 1e-6)
    b = _fused(batch, 1e-6)
    its = [(max(i["iters"] for i in p), max(i["iters"] for i in d)) for p, d in zip(b[1], b[2])]
    print(f"[solve_bounds] 3D iterations (primal, dual) per cell {its}", flush=True)
    _same(a, b)


@pytest.mark.parametrize("mode", ["gap", "timing"])
def test_fused_after_both_stop_paths(mode):
    """Under the gap rule and with per-kernel timing the bound passes wait for
    both sides (cross-stream lockstep, direct launches): still the separate
    calls' results, also on a second call (looser tolerance, fewer iterations)
    into the same buffers."""
    H = _H()
    cells = [homgen.square_inclusion_cell(2, side=0.25 + 0.15 * i, rho_in=30.0 * (i + 1)) for i in range(3)]
    batch = _batch(H, cells, 13, precision="mixed")
    if mode == "gap":
        batch.set_stop("gap", 1e-2, 1.0, 100.0)
    else:
        batch.set_timing(True)
    for tol in (1e-8, 1e-4):
        a = _separate(batch, tol)
        b = _fused(batch, tol)
        _same(a, b)


def test_fused_rejects_too_few_loads():
    H = _H()
    from paper_1404_3614_amd import _lib as L
    batch = _batch(H, [homgen.square_inclusion_cell(2)], 13, precision="mixed", max_loads=1)
    with pytest.raises(H.HomError):
        batch.solve_bounds(tol=1e-6)
    assert L.load().hom_batch_solve_bounds(None, None, None, 1e-6, 10, None, None, None, None, None) == L.HOM_E_INVALID


@pytest.mark.parametrize("launch", ["graph", "streams"])
def test_group_fused_equals_separate(launch):
    """hom_group_solve_bounds over three batches (2D N = 13 and N = 41, 3D
    N = 41) against hom_group_solve_pair followed by hom_batch_bounds: the
    same bounds, iterations and fields to the bit in both launch modes."""
    import torch
    H = _H()
    b2a = _batch(H, [homgen.square_inclusion_cell(2, side=0.2 + 0.1 * i, rho_in=10.0 * 4 ** i) for i in range(3)], 13)
    b2b = _batch(H, [homgen.square_inclusion_cell(2, side=0.45, rho_in=300.0),
                     homgen.square_inclusion_cell(2, side=0.3, rho_in=5.0)], 41)
    b3 = _batch(H, [homgen.sphere_cell(seed=90 + i, n=5 + 5 * i, rho=10.0 ** (1 + i)) for i in range(2)], (41, 41, 41))
    grp = H.Group([b2a, b2b, b3])
    grp.set_launch(launch)

    def run(fused):
        out = grp.solve_bounds(tol=1e-6, maxit=3000, fused=fused)
        fields = [[t.cpu() for f in b._fields(dual, b.d) for t in f] for b in grp.batches for dual in (False, True)]
        return out, fields

    a, fa = run(False)
    b, fb = run(True)
    for ba, bb in zip(a, b):
        for ra, rb in zip(ba, bb):
            for k in KEYS:
                assert np.array_equal(ra[k], rb[k]), k
            for side in ("info_primal", "info_dual"):
                assert [i["iters"] for i in ra[side]] == [i["iters"] for i in rb[side]]
    print(f"[solve_bounds] group {launch} iterations "
          f"{[[(max(i['iters'] for i in r['info_primal']), max(i['iters'] for i in r['info_dual'])) for r in bb] for bb in b]}",
          flush=True)
    for la, lb in zip(fa, fb):
        for u, v in zip(la, lb):
            assert torch.equal(u, v)
