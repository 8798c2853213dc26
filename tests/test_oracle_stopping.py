"""Pins for oracle.stopping: the energy recurrence of CG, the spectrum bound mu
and the Gauss-Radau bound on the remaining energy.

S1 energy recurrence e0 - sum alpha gamma = double-grid quadrature of the
   energy (the bound diagonal) at several iterates, and = e0 - <x, b + r>.
S2 the phases' eigenvalue range, and the smallest coefficient eigenvalue over
   the doubled grid, bound the spectrum of the dense Galerkin matrix (Lemma
   Ga_full, no doubled grid).
S3 Gauss-Radau bound >= exact remaining energy (from the dense direct solve)
   at every iterate, <= gamma / mu; on random SPD matrices with the exact
   smallest eigenvalue as well.
S4 the guaranteed rule stops at the first iterate whose bound meets etol, with
   the energy within etol of the converged one; the heuristic rule ends near
   the converged energy on a smooth case.
S5 the gap rule (primal and dual in lockstep): against the exact minimum
   energies of the dense direct solves, each side's final bound is within
   theta times the converged discretisation gap D*, the lower bound on D* it
   stopped on is one, the enclosure |E|^4 / V <= E . A_H E <= U holds, and
   the partner values it read are those of the previous chunk's last iterate
   (brute force over the recorded histories).
"""
import numpy as np
import pytest

import homgen
from oracle import dense, galerkin as ga, stopping as stp


def _aniso_rects(seed=7):
    rng = np.random.default_rng(seed)
    c = homgen.Inclusions(d=2, Y=np.array([1.0, 1.3]), A0=homgen.random_spd(rng, 2, 0.5, 2.0))
    c.add("rect", [0.2, -0.1], [0.3, 0.5], homgen.random_spd(rng, 2, 1.0, 30.0))
    c.add("rect", [-0.3, 0.45], [0.25, 0.2], homgen.random_spd(rng, 2, 1.0, 30.0))
    return c


CASES = {
    "square": (lambda: homgen.square_inclusion_cell(rho_in=20.0), (9, 9)),
    "aniso": (_aniso_rects, (7, 9)),
}


@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
@pytest.mark.parametrize("name", list(CASES))
def test_S1_energy_recurrence_is_the_quadrature(name, dual):
    make, N = CASES[name]
    prob = ga.make_problem(make(), N)
    coef = prob.Btil if dual else prob.Atil
    for E in (np.array([1.0, 0.0]), np.array([0.3, -1.1])):
        for k in (0, 1, 3, 8):
            res = stp.solve(prob, E, dual=dual, tol=1e-30, rule=None, maxit=k)
            assert res.iters == k
            quad = ga.energy_matrix(coef, [res.x], [E])[0, 0]
            assert abs(res.energy[-1] - quad) <= 1e-12 * quad
            assert abs(stp.energy_of(prob, res.x, E, dual) - quad) <= 1e-12 * quad
        # non-increasing along the iterates (CG minimises over growing Krylov spaces)
        res = stp.solve(prob, E, dual=dual, tol=1e-12, rule=None)
        assert np.all(np.diff(res.energy) <= 1e-15 * res.energy[0])


def _dense_K(prob, dual):
    Ah = prob.Bhat if dual else prob.Ahat
    K, _, _ = dense.dense_matrix(dense.ahat_lookup(Ah), prob.N, prob.Y, dual)
    return K


def phase_eig_range(cell):
    """Smallest and largest eigenvalue over the phases of a cell."""
    mats = [cell.A0] + list(cell.A)
    ev = np.concatenate([np.linalg.eigvalsh(np.asarray(A, float)) for A in mats])
    return float(ev.min()), float(ev.max())


@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
@pytest.mark.parametrize("name", list(CASES))
def test_S2_mu_bounds_the_dense_spectrum(name, dual):
    make, N = CASES[name]
    cell = make()
    prob = ga.make_problem(cell, (5, 7))
    K = _dense_K(prob, dual)
    lam = np.linalg.eigvalsh(K)
    # the coefficient's own eigenvalue range bounds the Galerkin spectrum
    a_min, a_max = phase_eig_range(cell)
    lo = 1.0 / a_max if dual else a_min
    assert lo <= lam[0] * (1 + 1e-12)
    assert lam[-1] <= (1.0 / a_min if dual else a_max) * (1 + 1e-12)
    # the doubled-grid minimum bounds it too, though Gibbs oscillations of the
    # truncated series can make it vacuous (negative) at high contrast
    mu = stp.spectrum_lower_bound(prob.Btil if dual else prob.Atil)
    assert mu <= lam[0] * (1 + 1e-12)


def _exact_remaining(prob, E, dual):
    """energy(x*) from the dense direct solve and the dense energy sum."""
    Ah = prob.Bhat if dual else prob.Ahat
    f = dense.ahat_lookup(Ah)
    xs = dense.dense_solve(f, prob.N, prob.Y, E, dual=dual)
    return dense.dense_energy(f, prob.N, [xs], [E])[0, 0]


@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_S3_radau_bound_dominates_the_remaining_energy(dual):
    cell = _aniso_rects(11)
    prob = ga.make_problem(cell, (5, 7))
    E = np.array([0.6, 0.8])
    e_star = _exact_remaining(prob, E, dual)
    a_min, a_max = phase_eig_range(cell)
    mu = 1.0 / a_max if dual else a_min
    res = stp.solve(prob, E, dual=dual, tol=1e-13, rule=None, mu=mu)
    rem = np.array(res.energy) - e_star
    rad = np.array(res.radau)
    g = np.array(res.gamma)
    mask = rem > 1e-13 * e_star          # above the rounding of the two energies
    assert mask.sum() >= 5
    assert np.all(rad[mask] >= rem[mask] * (1 - 1e-9))
    assert np.all(rad <= g / mu * (1 + 1e-12))


def test_S3_radau_bound_on_random_spd_matrices():
    rng = np.random.default_rng(5)
    for trial in range(30):
        n = int(rng.integers(10, 60))
        ev = np.exp(rng.uniform(0.0, np.log([10.0, 1e3, 1e5][trial % 3]), n))
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = (Q * ev) @ Q.T
        b = rng.standard_normal(n)
        xs = np.linalg.solve(A, b)
        e_star = -b @ xs                 # energy x^T A x - 2 b^T x at the solution, e0 = 0
        # mu below the spectrum, and at its exact bottom, where the bound turns tight
        # and the rounding of the recurrences (loss of orthogonality at high
        # condition numbers) shows at the 1e-4 level
        for mu, slack in ((0.3 * ev.min(), 1e-9), (ev.min(), 1e-3)):
            res = stp.cg_energy(lambda v: A @ v, b, 0.0, 1.0, tol=1e-12, rule=None, mu=mu, maxit=3 * n)
            rem = np.array(res.energy) - e_star
            rad = np.array(res.radau)
            mask = rem > 1e-10 * abs(e_star)
            assert np.all(rad[mask] >= rem[mask] * (1 - slack)), (trial, mu)


@pytest.mark.parametrize("dual", [False, True], ids=["primal", "dual"])
def test_S4_guaranteed_rule_accuracy_and_savings(dual):
    cell = homgen.square_inclusion_cell(rho_in=50.0)
    prob = ga.make_problem(cell, (9, 9))
    E = np.array([1.0, 0.0])
    a_min, a_max = phase_eig_range(cell)
    mu = 1.0 / a_max if dual else a_min
    ref = stp.solve(prob, E, dual=dual, tol=1e-13, rule=None)
    for etol in (1e-4, 1e-7, 1e-10):
        res = stp.solve(prob, E, dual=dual, tol=1e-30, rule="guaranteed", etol=etol, mu=mu)
        assert res.status == "energy"
        excess = res.energy[-1] - ref.energy[-1]
        assert -1e-13 * ref.energy[-1] <= excess <= etol * res.energy[-1]
        # the first iterate whose bound meets etol
        assert res.radau[-1] <= etol * res.energy[-1]
        assert all(r > etol * e for r, e in zip(res.radau[:-1], res.energy[:-1]))
    # heuristic rule: ends, and with the energy near the converged one on this smooth case
    res = stp.solve(prob, E, dual=dual, tol=1e-30, rule="heuristic", etol=1e-8)
    assert res.status == "energy"
    assert res.energy[-1] - ref.energy[-1] <= 1e-7 * ref.energy[-1]


def _pair_case(rho=50.0, N=(9, 9)):
    cell = homgen.square_inclusion_cell(rho_in=rho)
    prob = ga.make_problem(cell, N)
    a_min, a_max = phase_eig_range(cell)
    return prob, (a_min, 1.0 / a_max)


@pytest.mark.parametrize("E", [np.array([1.0, 0.0]), np.array([0.6, -0.8]), np.array([2.0, 1.0])],
                         ids=["e1", "unit_oblique", "norm_sqrt5"])
@pytest.mark.parametrize("theta", [0.1, 1e-3])
def test_S5_gap_rule_final_bounds_within_theta_of_the_gap(E, theta):
    prob, mu = _pair_case()
    U_star = _exact_remaining(prob, E, False)       # min primal energy: E . Abar E of the minimiser
    V_star = _exact_remaining(prob, E, True)        # min dual energy for J = E
    n4 = float(E @ E) ** 2
    D_star = U_star - n4 / V_star
    P, D, dlow = stp.solve_pair_gap(prob, E, tol=1e-30, theta=theta, chunk=8, mu=mu)
    assert P.status == "gap" and D.status == "gap"
    U, V = P.energy[-1], D.energy[-1]
    # guaranteed enclosure of E . A_H E by the iterates and by the limits
    assert n4 / V <= n4 / V_star * (1 + 1e-12) and U_star <= U * (1 + 1e-12)
    assert 0 < D_star
    # the stops used true lower bounds on D*, and each side's error is within theta D*
    assert 0 < dlow[0] <= D_star * (1 + 1e-9) and 0 < dlow[1] <= D_star * (1 + 1e-9)
    assert U - U_star <= theta * D_star * (1 + 1e-9)
    assert n4 / V_star - n4 / V <= theta * D_star * (1 + 1e-9)
    # no later than the residual rule at 1e-10
    ref_p = stp.solve(prob, E, dual=False, tol=1e-10, rule=None)
    ref_d = stp.solve(prob, E, dual=True, tol=1e-10, rule=None)
    assert P.i <= ref_p.iters and D.i <= ref_d.iters


def test_S5_gap_rule_reads_the_previous_chunk():
    """Brute force: replay the recorded histories and check that every stop
    decision used the partner state of iterate c m - 1 (c = i // m >= 1; during
    the first chunk nothing stops), and that no earlier iterate met the rule."""
    prob, mu = _pair_case(rho=200.0, N=(11, 11))
    E = np.array([1.0, 0.0])
    theta, m = 1e-2, 5
    P, D, dlow = stp.solve_pair_gap(prob, E, tol=1e-30, theta=theta, chunk=m, mu=mu)
    runs = (P, D)

    def low(V, RV):
        return 1.0 / V, (RV / (V * (V - RV)) if V > RV else np.inf)

    for k, rk in enumerate(runs):
        other = runs[1 - k]
        for i in range(rk.i + 1):
            c = i // m
            if c == 0:
                assert i != rk.i
                continue
            j = min(c * m - 1, other.i)
            if k == 0:
                U, RU = rk.energy[i], rk.radau[i]
                L, RL = low(other.energy[j], other.radau[j])
                own = RU
            else:
                U, RU = other.energy[j], other.radau[j]
                L, RL = low(rk.energy[i], rk.radau[i])
                own = RL
            dl = (U - RU) - (L + RL)
            hit = dl > 0 and own <= theta * dl
            assert hit == (i == rk.i), (k, i)
        assert abs(dlow[k] - dl) <= 1e-15 * abs(dl)
