"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (derived from the arithmetic of each mode):
  * operator, FP64 mode: 1e-12 relative (rounding of two FFT passes of length <= 625);
  * operator, mixed mode: 2e-6 relative (FP32 FFTs: ~ eps32 * log2(M^d) * a few);
  * bounds, FP64 mode, CG to 1e-10: 1e-9 relative (the bound error is quadratic in
    the field error, Lemma estimates, so 1e-10 residual gives ~1e-18 x contrast);
  * bounds, mixed mode: 1e-6 relative (the required accuracy; the field error of
    FP32 matvecs enters the bound squared).
Relative bound error = max_ab |X_gpu - X_ref|_ab / ||X_ref||_2 for X in {Abar, Bbar^-1}.
"""
import json
import os

import numpy as np
import pytest

import homgen
from oracle import galerkin as ga, spectral as sp

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reference_bounds.json")


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def relerr(X, R):
    return float(np.abs(np.asarray(X) - np.asarray(R)).max() / np.linalg.norm(np.asarray(R), 2))


def rand_field(d, N, Y, dual, rng):
    u = rng.standard_normal((d,) + tuple(N))
    xh = sp.dft_nd(u, d)
    G = sp.proj_J(N, np.array(Y)) if dual else sp.proj_E(N, np.array(Y))
    return sp.apply_blockdiag(G, xh)


def aniso_squares(seed=1):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


CASES_OP = [
    ("c1", lambda: homgen.square_inclusion_cell(), (13, 13)),
    ("pix", lambda: homgen.pixel_cell(seed=5, P=25, values=(1.0, 30.0)), (41, 41)),
    ("aniso2d_rect", aniso_squares, (13, 41)),
    ("n3", lambda: homgen.square_inclusion_cell(rho_in=4.0), (3, 3)),
    ("sph3d", lambda: homgen.sphere_cell(seed=3, n=4, anisotropic=True), (5, 13, 5)),
    ("sph3d_iso", lambda: homgen.sphere_cell(seed=9, n=6, anisotropic=False), (13, 13, 13)),
    # M = 81 on every axis, isotropic: the mixed operator runs the 3D plane pass
    ("sph3d_41", lambda: homgen.sphere_cell(seed=12, n=10, anisotropic=False, rho=10.0), (41, 41, 41)),
]


@pytest.mark.parametrize("name,mk,N", CASES_OP, ids=[c[0] for c in CASES_OP])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_operator_matches_oracle(name, mk, N, prec, dual):
    H = _H()
    import torch
    from layout import field_from_spectrum
    cell = mk()
    d = cell.d
    pb = H.problem_from_cell(cell, N, precision=prec)
    op = ga.make_problem(cell, N)
    rng = np.random.default_rng(17)
    xh = rand_field(d, N, cell.Y, dual, rng)
    c = field_from_spectrum(xh, d, N, cell.Y, dual)
    y = pb.apply(torch.tensor(c, dtype=torch.complex128, device="cuda"), dual).cpu().numpy()
    G = sp.proj_J(N, np.array(cell.Y)) if dual else sp.proj_E(N, np.array(cell.Y))
    yo = sp.apply_blockdiag(G, ga.ga_apply(op.Btil if dual else op.Atil, xh, N))
    co = field_from_spectrum(yo, d, N, cell.Y, dual)
    err = np.abs(y - co).max() / np.abs(co).max()
    assert err < (1e-12 if prec == "fp64" else 2e-6), err


CASES_B = [
    ("c1", lambda: homgen.square_inclusion_cell(), 13),
    ("pix2d", lambda: homgen.pixel_cell(seed=11, P=25, values=(1.0, 100.0)), 41),
    ("aniso2d", aniso_squares, (13, 41)),
    ("sph3d_aniso", lambda: homgen.sphere_cell(seed=4, n=5, anisotropic=True), 13),
    ("sph3d_nonuniform", lambda: homgen.sphere_cell(seed=6, n=4, anisotropic=False, rho=50.0), (13, 5, 41)),
]


@pytest.mark.parametrize("name,mk,N", CASES_B, ids=[c[0] for c in CASES_B])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bounds_match_oracle(name, mk, N, prec):
    H = _H()
    cell = mk()
    pb = H.problem_from_cell(cell, N, precision=prec)
    b = pb.solve_bounds(tol=1e-10 if prec == "fp64" else 1e-8)
    ob = ga.bounds(ga.make_problem(cell, N), tol=1e-11)
    tol = 1e-9 if prec == "fp64" else 1e-6
    assert relerr(b["A_up"], ob["A_up"]) < tol
    assert relerr(b["A_low"], ob["A_low"]) < tol
    assert all(i["status"] == 0 for i in b["info_primal"] + b["info_dual"])


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


GOLDEN_CELLS = {
    "C1": (lambda: homgen.square_inclusion_cell(d=2, side=0.5, rho_in=10.0), 13),
    "C2": (lambda: homgen.pixel_cell(1404002, P=125, values=(1.0, 100.0)), 313),
    "C3a": (lambda: homgen.sphere_cell(1404003, n=20, anisotropic=False, rho=10.0), 41),
    "C3b": (lambda: homgen.sphere_cell(1404003, n=20, anisotropic=True), 41),
}


@pytest.mark.parametrize("cfg", list(GOLDEN_CELLS))
@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-10, 1e-9), ("mixed", 1e-6, 1e-6)])
def test_configs_match_golden(cfg, prec, tol, bar):
    """Full-size configurations, in the launch configuration the benchmark uses."""
    H = _H()
    ref = _golden()[cfg]
    mk, N = GOLDEN_CELLS[cfg]
    pb = H.problem_from_cell(mk(), N, precision=prec)
    b = pb.solve_bounds(tol=tol)
    assert relerr(b["A_up"], ref["A_up"]) < bar
    assert relerr(b["A_low"], ref["A_low"]) < bar
    # Loewner chain of Lemma bounds and Voigt-Reuss (Remark Aeff_spd)
    for X, Yv in ((np.array(ref["reuss"]), b["A_low"]), (b["A_low"], b["A_up"]), (b["A_up"], np.array(ref["voigt"]))):
        assert np.linalg.eigvalsh(0.5 * (Yv - X + (Yv - X).T)).min() > -1e-9 * np.abs(Yv).max()


@pytest.mark.parametrize("d,rho,N", [(2, 10.0, 13), (2, 1e3, 41), (3, 10.0, 13)])
def test_laminate_closed_form_on_gpu(d, rho, N):
    H = _H()
    cell = homgen.laminate_cell(d=d, h=0.5, rho=rho)
    b = H.problem_from_cell(cell, N, precision="fp64").solve_bounds(tol=1e-11)
    arith, harm = 0.5 + 0.5 * rho, 1.0 / (0.5 + 0.5 / rho)
    for a in range(1, d):
        assert abs(b["A_up"][a, a] - arith) < 1e-11 * arith
    assert abs(b["A_low"][0, 0] - harm) < 1e-11 * harm


@pytest.mark.parametrize("d,N", [(2, 13), (3, 5)])
def test_homogeneous_takes_no_iteration(d, N):
    H = _H()
    A0 = np.eye(d) * 2.0 + 0.3 * (np.ones((d, d)) - np.eye(d))
    cell = homgen.homogeneous_cell(d, A0)
    b = H.problem_from_cell(cell, N, precision="mixed").solve_bounds(tol=1e-8)
    np.testing.assert_allclose(b["A_up"], A0, atol=1e-12)
    np.testing.assert_allclose(b["A_low"], A0, atol=1e-12)
    assert all(i["iters"] == 0 for i in b["info_primal"] + b["info_dual"])


def test_rotation_identity_dual_path_on_gpu():
    # 2D: Bbar(A) = R Abar(R^T A^-1 R) R^T (G^J = R G^E R^T), run through both GPU paths
    H = _H()
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    cell = aniso_squares(4)
    rot = homgen.Inclusions(d=2, Y=cell.Y, A0=R.T @ np.linalg.inv(cell.A0) @ R)
    for k, c, s, A in zip(cell.kind, cell.center, cell.size, cell.A):
        rot.add(k, c, s, R.T @ np.linalg.inv(A) @ R)
    b = H.problem_from_cell(cell, 41, precision="fp64").solve_bounds(tol=1e-11)
    r = H.problem_from_cell(rot, 41, precision="fp64").solve_bounds(tol=1e-11)
    assert relerr(b["B_up"], R @ r["A_up"] @ R.T) < 1e-10


def test_warm_start_from_solution_and_aliasing():
    H = _H()
    cell = homgen.pixel_cell(seed=2, P=25, values=(1.0, 50.0))
    pb = H.problem_from_cell(cell, 41, precision="fp64")
    x, info = pb.solve(False, tol=1e-10)
    assert info[0]["iters"] > 10
    x2, info2 = pb.solve(False, x0=x, tol=1e-9, out=x)   # x0 aliases the output
    assert all(i["iters"] <= 1 for i in info2)


def test_unconverged_iterate_still_gives_guaranteed_bounds():
    H = _H()
    cell = homgen.pixel_cell(seed=12, P=25, values=(1.0, 100.0))
    pb = H.problem_from_cell(cell, 41, precision="mixed")
    xp, ip = pb.solve(False, tol=1e-12, maxit=3, allow_not_converged=True)
    xd, idl = pb.solve(True, tol=1e-12, maxit=3, allow_not_converged=True)
    assert all(i["status"] == 1 for i in ip + idl)      # HOM_NOT_CONVERGED
    b = pb.bounds(xp, xd)
    ob = ga.bounds(ga.make_problem(cell, 41), tol=1e-11)
    # any admissible field gives Abar >= A_H,N and Bbar^-1 <= ...: here against the converged Ga bounds
    assert np.linalg.eigvalsh(b["A_up"] - ob["A_up"]).min() > -1e-10
    assert np.linalg.eigvalsh(ob["A_low"] - b["A_low"]).min() > -1e-10


def test_not_spd_is_reported():
    H = _H()
    cell = homgen.Inclusions(d=2, Y=np.ones(2), A0=np.eye(2))
    cell.add("rect", [0.0, 0.0], [0.5, 0.5], -3.0 * np.eye(2))
    pb = H.problem_from_cell(cell, 13, precision="fp64")
    with pytest.raises(H.HomError) as e:
        pb.solve(False, tol=1e-10)
    # breakdown <p, C p> <= 0 (HOM_E_NOT_SPD), or a non-finite residual (HOM_E_INVALID)
    assert e.value.status in (-3, -1)


def test_deterministic_and_graph_equals_eager(monkeypatch):
    H = _H()
    cell = homgen.sphere_cell(seed=8, n=5, anisotropic=True)
    pb = H.problem_from_cell(cell, 13, precision="mixed")
    a, _ = pb.solve(True, tol=1e-8)
    b, _ = pb.solve(True, tol=1e-8)
    monkeypatch.setenv("HOM_NO_GRAPH", "1")
    c, _ = pb.solve(True, tol=1e-8)
    for u, v, w in zip(a, b, c):
        assert bool((u == v).all()) and bool((u == w).all())


def test_plane_pass_is_bitwise_the_separate_passes(monkeypatch):
    """3D, N = 41 on every axis (M = 81), isotropic, mixed precision: the plane
    pass (middle, column and middle passes in one kernel, HOM_NO_PLANE unset)
    runs the FP32 operations of the three separate passes in their order, so
    operator applications, iteration counts, fields and bounds are the same to
    the bit; the per-pass profile shows no middle pass."""
    H = _H()
    import torch
    from layout import field_from_spectrum
    N = (41, 41, 41)
    cells = [homgen.sphere_cell(seed=60 + i, n=6 + 6 * i, anisotropic=False, rho=10.0 ** (1 + i)) for i in range(3)]
    rng = np.random.default_rng(29)
    x = torch.tensor(field_from_spectrum(rand_field(3, N, cells[0].Y, False, rng), 3, N, cells[0].Y, False),
                     dtype=torch.complex128, device="cuda")

    def run():
        st = torch.cuda.Stream()
        probs = [H.problem_from_cell(c, N, precision="mixed", stream=st) for c in cells]
        batch = H.Batch(probs)
        fp, ip, fd, idl = batch.solve_pair(tol=1e-6)
        out = batch.bounds(fp, fd)
        for i, r in enumerate(out):
            r.update(info_primal=ip[i], info_dual=idl[i], fields_primal=[t.cpu() for t in fp[i]],
                     fields_dual=[t.cpu() for t in fd[i]])
        y = probs[0].apply(x, False)                                    # one load: two packs
        x2, i2 = probs[1].solve(True, E=np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]), tol=1e-6)  # three packs
        prof = batch.profile_passes(False, 3, reps=2)
        torch.cuda.synchronize()
        return out, (y.cpu(), [t.cpu() for t in x2], [i["iters"] for i in i2]), prof

    monkeypatch.delenv("HOM_NO_PLANE", raising=False)
    a, ya, pa = run()
    monkeypatch.setenv("HOM_NO_PLANE", "1")
    b, yb, pb_ = run()
    print(f"[plane] profile plane {pa} separate {pb_}", flush=True)
    assert pa["mid_inv"] == 0 and pa["mid_fwd"] == 0 and pa["apply"] > 0
    assert pb_["mid_inv"] > 0 and pb_["mid_fwd"] > 0
    assert torch.equal(ya[0], yb[0]) and ya[2] == yb[2]
    for u, v in zip(ya[1], yb[1]):
        assert torch.equal(u, v)
    for ra, rb in zip(a, b):
        for key in ("info_primal", "info_dual"):
            assert [i["iters"] for i in ra[key]] == [i["iters"] for i in rb[key]]
        for key in ("fields_primal", "fields_dual"):
            for u, v in zip(ra[key], rb[key]):
                assert torch.equal(u, v)
        assert np.array_equal(ra["A_up"], rb["A_up"]) and np.array_equal(ra["A_low"], rb["A_low"])


def _voxels(P, seed):
    rng = np.random.default_rng(seed)
    return homgen.Pixels(d=3, Y=np.array([1.0, 0.8, 1.2]), phase=rng.integers(0, 3, size=P),
                         phase_A=np.stack([homgen.random_spd(rng, 3, 1.0, 5.0) for _ in range(3)]))


def test_setup_coefficients_match_oracle():
    # device Fourier coefficients (hom_coef_inclusions / hom_coef_pixels) against the oracle's
    H = _H()
    from oracle import coefficients as co
    for cell, N in ((homgen.sphere_cell(seed=1, n=7, anisotropic=True), (5, 13, 13)),
                    (homgen.pixel_cell(seed=4, P=25, values=(2.0, 7.0)), (13, 41)),
                    (aniso_squares(2), (13, 13)),
                    # images of 2^k pixels: the image transform has radix-2/4 stages
                    (homgen.pixel_cell(seed=6, P=16, values=(1.0, 9.0)), (13, 23)),
                    (_voxels((8, 4, 10), seed=7), (5, 13, 5))):
        M = tuple(2 * n - 1 for n in N)
        Ah, Bh, nc = H.coef_from_cell(cell, N)
        ref = co.fourier_coefficients(cell, M)
        refB = co.fourier_coefficients(cell, M, inverse=True)
        d = cell.d
        comp = [(0, 0)] if nc == 1 else ([(0, 0), (1, 1), (0, 1)] if d == 2 else
                                         [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)])
        for c, (i, j) in enumerate(comp):
            assert np.abs(Ah[c].cpu().numpy() - ref[i, j]).max() < 1e-13 * max(1, np.abs(ref).max())
            assert np.abs(Bh[c].cpu().numpy() - refB[i, j]).max() < 1e-13 * max(1, np.abs(refB).max())


def test_batch_equals_single_problem_solves():
    # lockstep batching runs the same per-problem arithmetic: results are bitwise equal
    H = _H()
    import torch
    cells = [homgen.pixel_cell(seed=30 + i, P=25, values=(1.0, 20.0 + 30 * i)) for i in range(3)]
    st = torch.cuda.Stream()
    probs = []
    for c in cells:
        Ah, Bh, nc = H.coef_from_cell(c, (41, 41))
        probs.append(H.Problem(2, (41, 41), (1.0, 1.0), Ah, Bh, precision="mixed", ncoef=nc, max_loads=2, stream=st))
    batch = H.Batch(probs)
    out = batch.solve_bounds(tol=1e-8)
    for p, c, b in zip(probs, cells, out):
        single = p.solve_bounds(tol=1e-8)
        assert np.array_equal(single["A_up"], b["A_up"]) and np.array_equal(single["A_low"], b["A_low"])
        assert [i["iters"] for i in single["info_primal"]] == [i["iters"] for i in b["info_primal"]]
        ob = ga.bounds(ga.make_problem(c, 41), tol=1e-11)
        assert relerr(b["A_up"], ob["A_up"]) < 1e-6 and relerr(b["A_low"], ob["A_low"]) < 1e-6


def test_batch_3d_mixed_contrast():
    H = _H()
    import torch
    st = torch.cuda.Stream()
    cells = [homgen.sphere_cell(seed=40 + i, n=4 + i, anisotropic=(i == 1)) for i in range(3)]
    nc = 6
    probs = []
    for c in cells:
        Ah, Bh, _ = H.coef_from_cell(c, (13, 13, 13), ncoef=nc)
        probs.append(H.Problem(3, (13, 13, 13), (1.0, 1.0, 1.0), Ah, Bh, precision="fp64", ncoef=nc, stream=st))
    out = H.Batch(probs).solve_bounds(tol=1e-10)
    for c, b in zip(cells, out):
        ob = ga.bounds(ga.make_problem(c, 13), tol=1e-11)
        assert relerr(b["A_up"], ob["A_up"]) < 1e-9 and relerr(b["A_low"], ob["A_low"]) < 1e-9


def test_update_coefficients_matches_fresh_setup_and_timing_counts():
    H = _H()
    import torch
    st = torch.cuda.Stream()
    cells = [homgen.pixel_cell(seed=50 + i, P=25, values=(1.0, 10.0 + 40 * i)) for i in range(2)]
    coefs = [H.coef_from_cell(c, (41, 41)) for c in cells]
    probs = [H.Problem(2, (41, 41), (1.0, 1.0), *coefs[i][:2], precision="mixed", ncoef=1, max_loads=2, stream=st)
             for i in range(2)]
    batch = H.Batch(probs)
    batch.set_timing(True)
    first = batch.solve_bounds(tol=1e-8)
    ms, cnt = batch.get_timing()
    assert cnt["first"] == cnt["apply"] == cnt["last"] > 0 and ms["apply"] > 0
    batch.set_timing(False)
    # swap the coefficients between the two problems and solve again with the same batch
    probs[0].update_coefficients(*coefs[1][:2])
    probs[1].update_coefficients(*coefs[0][:2])
    swapped = batch.solve_bounds(tol=1e-8)
    assert np.array_equal(swapped[0]["A_up"], first[1]["A_up"])
    assert np.array_equal(swapped[1]["A_low"], first[0]["A_low"])


@pytest.mark.parametrize("d,N", [(2, 41), (2, 313), (3, 13)])
def test_batch_coefficient_update_equals_per_problem_setup(d, N):
    """hom_batch_update_coefficients sets up every cell in three launches where
    the specialised 2D set-up exists (cell by cell otherwise); the grid
    coefficients, and so the bounds, are bitwise those of single set-ups."""
    H = _H()
    import torch
    st = torch.cuda.Stream()
    n = 3
    if d == 2:
        cells = [homgen.pixel_cell(seed=70 + i, P=25, values=(1.0, 5.0 + 20 * i)) for i in range(2 * n)]
    else:
        cells = [homgen.sphere_cell(seed=70 + i, n=4, rho=5.0 + 10 * i) for i in range(2 * n)]
    NN = (N,) * d
    coefs = [H.coef_from_cell(c, NN) for c in cells]
    nc = coefs[0][2]
    assert all(c[2] == nc for c in coefs)
    probs = [H.Problem(d, NN, cells[i].Y, *coefs[i][:2], precision="mixed", ncoef=nc, max_loads=d, stream=st)
             for i in range(n)]
    batch = H.Batch(probs)
    batch.update_coefficients([coefs[n + i][:2] for i in range(n)])
    got = batch.solve_bounds(tol=1e-8)
    for i in range(n):
        ref = H.Problem(d, NN, cells[n + i].Y, *coefs[n + i][:2], precision="mixed", ncoef=nc, max_loads=d,
                        stream=st)
        rb = H.Batch([ref]).solve_bounds(tol=1e-8)[0]
        assert np.array_equal(got[i]["A_up"], rb["A_up"]) and np.array_equal(got[i]["A_low"], rb["A_low"]), i


def test_side_by_side_pair_equals_sequential_solves():
    # the dual on the library's second stream: same kernels, same reductions, so bitwise equal;
    # sequential solves reuse the same captured graphs afterwards
    H = _H()
    import torch
    st = torch.cuda.Stream()
    cells = [homgen.pixel_cell(seed=70 + i, P=25, values=(1.0, 15.0 + 25 * i)) for i in range(3)]
    probs = [H.problem_from_cell(c, (41, 41), precision="mixed", max_loads=2, stream=st) for c in cells]
    batch = H.Batch(probs)
    for rep in range(2):
        fp, ip, fd, idl = batch.solve_pair(tol=1e-8)
        sp, isp = batch.solve(False, tol=1e-8)
        sd, isd = batch.solve(True, tol=1e-8)
        for i in range(3):
            for l in range(2):
                assert bool((fp[i][l] == sp[i][l]).all()) and bool((fd[i][l] == sd[i][l]).all())
                assert ip[i][l]["iters"] == isp[i][l]["iters"] and idl[i][l]["iters"] == isd[i][l]["iters"]
                assert ip[i][l]["status"] == 0 and idl[i][l]["status"] == 0


def test_bandwidth_probe_copies_and_reports_a_rate():
    H = _H()
    import torch
    g = H.probe_copy_gbs(1 << 26, reps=3)
    print(f"[probe] copy of 64 MiB: {g:.0f} GB/s", flush=True)
    assert 100.0 < g < 20000.0
    from paper_1404_3614_amd import _lib as L
    src = torch.zeros(1024, dtype=torch.float32, device="cuda")
    gbs = L.C.c_double()
    for bad in ((src.data_ptr() + 4, src.data_ptr(), 1024, 1), (src.data_ptr(), src.data_ptr(), 1000, 1),
                (src.data_ptr(), src.data_ptr(), 1024, 0)):
        with pytest.raises(H.HomError):
            L.check(L.load().hom_probe_copy(L.C.c_void_p(bad[0]), L.C.c_void_p(bad[1]), bad[2], bad[3], None,
                                            L.C.byref(gbs)), "hom_probe_copy")
