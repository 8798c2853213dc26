"""Pins for oracle.galerkin / dense / gani against closed forms, invariants and
an independent dense formulation.

P1 homogeneous medium: the bounds equal A0 and CG takes no step.
P2 laminate: exact arithmetic/harmonic means in the directions where the
   Galerkin space contains the exact minimiser; GaNi duality on odd grids.
P3 dense Fourier-Galerkin system (Lemma Ga_full) versus the double-grid FFT route.
P4 Loewner chain, Voigt-Reuss, symmetry, monotonicity in N and in CG steps.
P5 2D rotation identity: the dual with A^{-1} is the rotated primal with A^{-1}.
P7 double-grid quadrature (Lemma integral_eval_double_grid) versus the dense sum.
P9 convergence of the guaranteed error; Hashin-Shtrikman window for the square.
"""
import numpy as np
import pytest

import homgen
from oracle import galerkin as ga, dense, gani
from oracle import coefficients as co
from oracle.spectral import freqs


def _spd_le(A, B, tol=1e-12):
    """A <= B in the Loewner order."""
    return np.linalg.eigvalsh(0.5 * ((B - A) + (B - A).T)).min() >= -tol * max(1.0, np.abs(B).max())


@pytest.mark.parametrize("d,A0", [(2, [[2.0, 0.5], [0.5, 1.0]]),
                                  (3, [[3.0, 0.2, 0.1], [0.2, 1.0, -0.3], [0.1, -0.3, 2.0]]),
                                  (2, [[5.0, 0.0], [0.0, 5.0]])])
def test_P1_homogeneous(d, A0):
    A0 = np.array(A0)
    prob = ga.make_problem(homgen.homogeneous_cell(d, A0), 5 if d == 3 else 7)
    b = ga.bounds(prob)
    np.testing.assert_allclose(b["A_up"], A0, atol=1e-13)
    np.testing.assert_allclose(b["A_low"], A0, atol=1e-13)
    assert max(b["iters_primal"] + b["iters_dual"]) == 0


@pytest.mark.parametrize("d,rho,N,Y", [(2, 10.0, 9, (1.0, 1.0)), (2, 1e3, 11, (1.0, 2.0)),
                                       (3, 10.0, 5, (1.0, 1.0, 1.0))])
def test_P2_laminate(d, rho, N, Y):
    Y = np.array(Y)
    h = 0.5 * Y[0]
    cell = homgen.laminate_cell(d=d, h=h, rho=rho, Y=Y)
    prob = ga.make_problem(cell, N)
    b = ga.bounds(prob)
    f = h / Y[0]
    arith = (1 - f) + f * rho
    harm = 1.0 / ((1 - f) + f / rho)
    # the transverse load has the exact minimiser 0 in E_N: Abar_22 = <a>
    for a in range(1, d):
        assert abs(b["A_up"][a, a] - arith) < 1e-12 * arith
    # the dual load along the layering normal has j = 0: (Bbar^{-1})_11 = harmonic mean
    assert abs(b["A_low"][0, 0] - harm) < 1e-12 * harm
    off = b["A_up"] - np.diag(np.diag(b["A_up"]))
    assert np.abs(off).max() < 1e-12
    assert b["A_up"][0, 0] >= harm - 1e-12
    assert b["A_low"][1, 1] <= arith + 1e-12
    assert _spd_le(b["A_low"], b["A_up"])


@pytest.mark.parametrize("rho,N", [(10.0, 9), (1e3, 13)])
def test_P2_laminate_gani_odd_duality_closed_form(rho, N):
    cell = homgen.laminate_cell(d=2, h=0.5, rho=rho)
    g = gani.gani_bounds(cell, N)
    a_k = co.point_values(cell, (N, N))[0, 0][:, 0]
    harmN = 1.0 / np.mean(1.0 / a_k)
    arithN = np.mean(a_k)
    np.testing.assert_allclose(g["A_HN"], np.diag([harmN, arithN]), atol=1e-10 * rho)
    np.testing.assert_allclose(np.linalg.inv(g["B_HN"]), np.diag([harmN, arithN]), atol=1e-10 * rho)


def _dense_vs_fft(cell, N, tol=1e-12):
    prob = ga.make_problem(cell, N)
    b = ga.bounds(prob, tol=1e-14)
    db = dense.dense_bounds(dense.ahat_lookup(prob.Ahat), dense.ahat_lookup(prob.Bhat), prob.N, prob.Y)
    scale = np.abs(db["A_up"]).max()
    assert np.abs(b["A_up"] - db["A_up"]).max() < tol * scale
    assert np.abs(b["A_low"] - db["A_low"]).max() < tol * scale
    d = prob.d
    for a in range(d):
        xf = dense.to_array(db["prim"][a], prob.N, d)
        assert np.abs(b["fields_primal"][a] - xf).max() < 1e-10 * max(1.0, np.abs(xf).max())
        jf = dense.to_array(db["dual"][a], prob.N, d)
        assert np.abs(b["fields_dual"][a] - jf).max() < 1e-10 * max(1.0, np.abs(jf).max())


@pytest.mark.parametrize("N", [5, 7])
def test_P3_dense_square_inclusion(N):
    _dense_vs_fft(homgen.square_inclusion_cell(rho_in=10.0), N)


def test_P3_dense_offcentre_anisotropic_2d_nonunit_cell():
    rng = np.random.default_rng(9)
    cell = homgen.Inclusions(d=2, Y=np.array([1.0, 1.7]), A0=homgen.random_spd(rng, 2))
    cell.add("rect", [0.21, -0.33], [0.3, 0.5], homgen.random_spd(rng, 2))
    cell.add("rect", [-0.3, 0.5], [0.2, 0.3], homgen.random_spd(rng, 2))
    _dense_vs_fft(cell, (7, 5))


def test_P3_dense_pixels():
    pix = homgen.pixel_cell(seed=3, P=5, values=(1.0, 20.0))
    _dense_vs_fft(pix, 5)


def test_P3_dense_3d_anisotropic_spheres():
    cell = homgen.sphere_cell(seed=4, n=4, anisotropic=True)
    _dense_vs_fft(cell, 5)


@pytest.mark.parametrize("cell", [homgen.pixel_cell(seed=8, P=9, values=(1.0, 50.0)),
                                  homgen.sphere_cell(seed=5, n=5, anisotropic=True)],
                         ids=["pixels2d", "spheres3d"])
def test_P4_invariants(cell):
    N = 9 if cell.d == 2 else 7
    prob = ga.make_problem(cell, N)
    b = ga.bounds(prob)
    voigt, reuss = ga.voigt_reuss(prob)
    for X in (b["A_up"], b["B_up"]):
        np.testing.assert_allclose(X, X.T, atol=1e-12 * np.abs(X).max())
    assert _spd_le(reuss, b["A_low"])
    assert _spd_le(b["A_low"], b["A_up"])
    assert _spd_le(b["A_up"], voigt)


def test_P4_monotone_in_N_square():
    # E_N is nested in E_N' for N < N' and the Ga bounds are exact energies
    cell = homgen.square_inclusion_cell(rho_in=10.0)
    ups, lows = [], []
    for N in (5, 7, 9, 11, 13, 15):
        b = ga.bounds(ga.make_problem(cell, N))
        ups.append(b["A_up"][0, 0])
        lows.append(b["A_low"][0, 0])
    assert all(u1 >= u2 - 1e-12 for u1, u2 in zip(ups, ups[1:]))
    assert all(l1 <= l2 + 1e-12 for l1, l2 in zip(lows, lows[1:]))


def test_P4_cg_energy_monotone_and_upper_bound_from_any_iterate():
    cell = homgen.pixel_cell(seed=2, P=9, values=(1.0, 100.0))
    prob = ga.make_problem(cell, 9)
    e1 = np.eye(2)[0]
    energies = []
    ga.solve(prob, e1, tol=1e-12, callback=lambda x: energies.append(
        ga.energy_matrix(prob.Atil, [x], [e1])[0, 0]))
    assert len(energies) > 5
    assert all(a >= b - 1e-12 for a, b in zip(energies, energies[1:]))
    assert energies[0] >= energies[-1]


def _rotate_cell_inverse(cell):
    """Cell with the phase coefficients replaced by R^T A^{-1} R (R = 90 deg rotation)."""
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    tr = lambda A: R.T @ np.linalg.inv(A) @ R
    if hasattr(cell, "phase"):
        return homgen.Pixels(d=2, Y=cell.Y, phase=cell.phase,
                             phase_A=np.stack([tr(A) for A in cell.phase_A]))
    out = homgen.Inclusions(d=2, Y=cell.Y, A0=tr(cell.A0))
    for k, c, s, A in zip(cell.kind, cell.center, cell.size, cell.A):
        out.add(k, c, s, tr(A))
    return out


@pytest.mark.parametrize("cell", [
    homgen.pixel_cell(seed=6, P=7, values=(1.0, 30.0)),
    homgen.Inclusions(d=2, Y=np.ones(2), A0=np.array([[1.5, 0.2], [0.2, 0.7]])).add(
        "rect", [0.1, -0.2], [0.4, 0.3], np.array([[8.0, -1.0], [-1.0, 3.0]]))],
    ids=["pixels", "anisotropic"])
def test_P5_rotation_identity_dual_equals_rotated_primal(cell):
    # In 2D G^J(k) = R G^E(k) R^T with R the rotation by 90 degrees, hence the dual
    # problem with A^{-1} is the primal problem with R^T A^{-1} R, rotated back.
    N = 7
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    b = ga.bounds(ga.make_problem(cell, N), tol=1e-13)
    rot = ga.bounds(ga.make_problem(_rotate_cell_inverse(cell), N), tol=1e-13)
    np.testing.assert_allclose(b["B_up"], R @ rot["A_up"] @ R.T, atol=1e-11 * np.abs(b["B_up"]).max())


def test_P5_two_phase_phase_swap():
    # isotropic two-phase: lower(1, rho) = rho * R Abar(rho, 1)^{-1} R^T
    rho = 25.0
    pix = homgen.pixel_cell(seed=10, P=7, values=(1.0, rho))
    swp = homgen.Pixels(d=2, Y=pix.Y, phase=pix.phase, phase_A=pix.phase_A[::-1].copy())
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    b = ga.bounds(ga.make_problem(pix, 9), tol=1e-13)
    s = ga.bounds(ga.make_problem(swp, 9), tol=1e-13)
    np.testing.assert_allclose(b["A_low"], rho * R @ np.linalg.inv(s["A_up"]) @ R.T, rtol=1e-10)


@pytest.mark.parametrize("d,N", [(2, (5, 7)), (3, (3, 5, 3))])
def test_P7_double_grid_quadrature_equals_dense_sum(d, N):
    rng = np.random.default_rng(12)
    cell = homgen.Inclusions(d=d, Y=np.ones(d) * 1.3, A0=homgen.random_spd(rng, d))
    cell.add("rect", rng.uniform(-0.5, 0.5, d), rng.uniform(0.1, 0.6, d), homgen.random_spd(rng, d))
    prob = ga.make_problem(cell, N)

    def rand_trig():
        # real field on the N grid -> Hermitian Fourier coefficients
        from oracle.spectral import dft_nd
        return dft_nd(rng.standard_normal((d,) + N), d)
    u, v = rand_trig(), rand_trig()
    M = prob.M
    uM, vM = ga.to_grid(u, M), ga.to_grid(v, M)
    quad = np.mean(np.sum(vM * np.einsum("ab...,b...->a...", prob.Atil, uM), axis=0))
    look = dense.ahat_lookup(prob.Ahat)
    ks = [np.array(k) for k in np.ndindex(*N)]
    fr = [freqs(n) for n in N]
    s = 0.0
    for li in ks:
        l = np.array([fr[a][li[a]] for a in range(d)])
        for ki in ks:
            k = np.array([fr[a][ki[a]] for a in range(d)])
            s += np.conj(v[(slice(None),) + tuple(li)]) @ look(l - k) @ u[(slice(None),) + tuple(ki)]
    assert abs(quad - s.real) < 1e-12 * abs(s)
    assert abs(s.imag) < 1e-12 * abs(s)


def test_P9_square_convergence_and_hashin_shtrikman():
    cell = homgen.square_inclusion_cell(rho_in=10.0)
    Ds = []
    for N in (5, 13, 41):
        b = ga.bounds(ga.make_problem(cell, N))
        # symmetry of the square: bounds proportional to I
        assert abs(b["A_up"][0, 0] - b["A_up"][1, 1]) < 1e-11
        assert abs(b["A_up"][0, 1]) < 1e-11
        # vf 0.25, contrast 10: HS lower 1.5143 <= A_H <= HS upper 2.3944
        f, r = 0.25, 10.0
        hs_lo = 1 + f / (1 / (r - 1) + (1 - f) / 2)
        hs_up = r + (1 - f) / (1 / (1 - r) + f / (2 * r))
        assert b["A_up"][0, 0] >= hs_lo
        assert b["A_low"][0, 0] <= hs_up
        Ds.append(b["D"][0, 0])
    assert Ds[0] > Ds[1] > Ds[2] > 0


def test_gani_odd_duality_and_ga_beats_gani_upper():
    pix = homgen.pixel_cell(seed=7, P=5, values=(1.0, 40.0))
    g = gani.gani_bounds(pix, 11)
    np.testing.assert_allclose(g["A_HN"], np.linalg.inv(g["B_HN"]), rtol=1e-9)
    b = ga.bounds(ga.make_problem(pix, 11))
    # Ga minimises the exact energy over the same space as the GaNi field
    assert _spd_le(b["A_up"], g["A_up"])
    assert _spd_le(g["A_low"], b["A_low"])
