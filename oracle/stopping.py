"""Energy of the CG iterates and stopping rules on it (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this package.

The Galerkin problems of oracle/galerkin.py minimise the energy
a(E + x, E + x) over x in E_N (primal; the dual minimises a^{-1}(J + j, J + j)
over J_N), and the minimum is the diagonal entry of the guaranteed bound
(Def. upper_lower_bounds).  CG minimises this energy over growing Krylov
spaces (Sec. 7.1), so every iterate gives a guaranteed, non-increasing bound,
and step i lowers the energy by alpha_i gamma_i (gamma_i = ||r_i||^2):

    energy(x) - energy(x*) = (x* - x)^T C (x* - x),   energy(x) = e0 - <x, b + r>,

e0 = E^T <A> E the energy of the zero field.  The Convergence-criteria remark
(Sec. 7.2) stops on the residual, with a tolerance picked so that the
algebraic error stays below the discretisation error; the rules here bound
that algebraic error in the energy itself:

* guaranteed: the Gauss-Radau quadrature of the Lanczos process behind CG
  bounds the remaining decrease (x* - x_i)^T C (x* - x_i) from above by
  gamma_i phi_i for any mu at or below the smallest eigenvalue of C, with
  phi_0 = 1/mu and phi_i = t / (mu t + gamma_i / gamma_{i-1}),
  t = phi_{i-1} - alpha_{i-1} (G. Meurant and P. Tichy, Numer. Algorithms,
  2019); gamma_i / mu bounds it as well.  The rule stops when the bound is
  below etol times the energy of the iterate.
* heuristic: the remaining decrease extrapolated as a geometric tail of the
  last four decrements (ratio rho = (d_{i-1} / d_{i-4})^{1/3}, remainder
  2 d_{i-1} rho / (1 - rho)), below etol times the energy of the iterate.

Both are extra exits beside the residual rule.  mu: the quadratic form of C
is the integral of v . A v over the cell, so the smallest eigenvalue a_min of
the coefficient bounds the spectrum of C from below (dual: 1 / a_max).  It is
also the mean over the doubled grid of v . A_M v (Lemma
integral_eval_double_grid), with sum |v|^2 the squared L2 norm of the field,
so the smallest eigenvalue of A_M over the grid points bounds it as well; the
truncated series oscillates near interfaces, which can make that second
bound vacuous (negative) at high contrast.

* gap (primal and dual together): for a load E, the primal energy U of the
  iterate is an upper bound on E . A_H E and L = |E|^4 / V, with V the dual
  energy of the dual iterate for J = E, a lower bound (V >= E . A_H^{-1} E and
  (E . E)^2 <= (E . A_H E)(E . A_H^{-1} E)); the converged difference
  D* = U* - L* is the discretisation gap of eq. approx_homog_with_error on
  this entry.  Following the Convergence-criteria remark (Sec. 7.2: the
  algebraic error should stay below the discretisation error), each side
  stops once the Gauss-Radau bound of its own remaining error is below theta
  times a guaranteed lower bound on D*: with R the primal bound (U - U* <= R)
  and R' = |E|^4 R_V / (V (V - R_V)) the bound on L* - L from the dual one
  (R' infinite unless V > R_V), D* >= (U - R) - (L + R'), and a side stops
  when its own R (R') is at most theta times that.  Both R and R' are valid
  at every iterate, so the partner's values may be old: the two solves
  advance in lockstep chunks of m iterations and each reads the other's
  (energy, bound) pair at the last iterate of the previous chunk (during the
  first chunk: its start energy with an infinite bound, so nothing stops
  there).  The rule is deterministic when the two run concurrently, and at
  the stop U - U* <= theta D* and L* - L <= theta D*.

Pinned by tests/test_oracle_stopping.py: the energy recurrence against the
double-grid quadrature of the bounds, mu against the eigenvalues of the
dense Galerkin matrix, the Gauss-Radau bound against the exact remaining
energy from a direct solve, and the stop decisions against their definitions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .galerkin import constant_field, ga_apply
from .spectral import apply_blockdiag, inner, proj_E, proj_J


def spectrum_lower_bound(coef_M):
    """Smallest eigenvalue of the symmetric coefficient over the doubled grid."""
    d = coef_M.shape[0]
    pts = np.moveaxis(coef_M.reshape(d, d, -1), -1, 0)
    return float(np.linalg.eigvalsh(pts)[:, 0].min())


@dataclass
class EnergyCG:
    x: np.ndarray
    iters: int
    status: str                                   # "residual", "energy" or "maxit"
    energy: list = field(default_factory=list)     # energy of iterate i from the recurrence
    radau: list = field(default_factory=list)      # Gauss-Radau bound on the remaining decrease of iterate i
    gamma: list = field(default_factory=list)


def operator(prob, dual):
    coef = prob.Btil if dual else prob.Atil
    G = proj_J(prob.N, prob.Y) if dual else proj_E(prob.N, prob.Y)

    def C(x):
        return apply_blockdiag(G, ga_apply(coef, x, prob.N))
    return C, coef


def zero_field_energy(prob, E, dual):
    """E^T <A> E (dual: with <A^{-1}>) from the zero frequency of the series."""
    E = np.asarray(E, float)
    Ah = prob.Bhat if dual else prob.Ahat
    A0 = Ah[(slice(None), slice(None)) + (0,) * prob.d].real
    return float(E @ A0 @ E)


def cg_energy(apply_C, b, e0, normE, tol=1e-8, rule="guaranteed", etol=1e-8, mu=0.0, maxit=20000):
    """Hestenes-Stiefel CG for C x = b from x0 = 0, tracking the energy
    e0 - sum alpha_i gamma_i and the Gauss-Radau bound of every iterate; the
    residual rule ||r|| <= tol normE and, beside it, the energy rule `rule`
    ("guaranteed", "heuristic" or None) at etol."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    gam = inner(r, r)
    energy, dec = e0, []
    out = EnergyCG(x=x, iters=0, status="maxit")
    phi = 1.0 / mu if mu > 0 else np.inf
    alpha_prev = gam_prev = None
    i = 0
    while True:
        # Gauss-Radau factor of iterate i
        if i > 0 and mu > 0:
            t = phi - alpha_prev
            ph = t / (mu * t + gam / gam_prev)
            phi = ph if (t > 0 and 0 < ph < 1.0 / mu) else 1.0 / mu
        out.energy.append(energy)
        out.radau.append(gam * phi)
        out.gamma.append(gam)
        if np.sqrt(gam) <= tol * normE:
            out.status = "residual"
            break
        if rule == "guaranteed" and gam * phi <= etol * energy:
            out.status = "energy"
            break
        if rule == "heuristic" and i >= 5:
            d1, d4 = dec[i - 1], dec[i - 4]
            if d1 >= 0 and d4 > 0:
                rho = (d1 / d4) ** (1.0 / 3.0)
                if rho < 0.99 and 2 * d1 * rho / (1 - rho) <= etol * energy:
                    out.status = "energy"
                    break
        if i >= maxit:
            break
        q = apply_C(p)
        pq = inner(p, q)
        if pq <= 0.0:
            raise FloatingPointError("operator not positive definite on the subspace")
        alpha = gam / pq
        x = x + alpha * p
        r = r - alpha * q
        gam_new = inner(r, r)
        dec.append(alpha * gam)
        energy -= alpha * gam
        p = r + (gam_new / gam) * p
        alpha_prev, gam_prev, gam = alpha, gam, gam_new
        i += 1
    out.x, out.iters = x, i
    return out


def solve(prob, E, dual=False, tol=1e-8, rule="guaranteed", etol=1e-8, mu=None, maxit=20000):
    """The primal (dual) Galerkin problem for load E by cg_energy.  mu: lower
    bound on the spectrum (default: spectrum_lower_bound of the coefficient)."""
    E = np.asarray(E, float)
    C, coef = operator(prob, dual)
    if mu is None:
        mu = spectrum_lower_bound(coef)
    b = -C(constant_field(E, prob.N))
    return cg_energy(C, b, zero_field_energy(prob, E, dual), float(np.linalg.norm(E)), tol, rule, etol, mu, maxit)


def energy_of(prob, x, E, dual=False):
    """e0 - <x, b + r>: the energy of a field from the operator (no recurrence)."""
    C, _ = operator(prob, dual)
    b = -C(constant_field(np.asarray(E, float), prob.N))
    r = b - C(x)
    return zero_field_energy(prob, E, dual) - float(np.real(inner(x, b + r)))


class _CGRun:
    """One Hestenes-Stiefel CG from x0 = 0 advanced an iteration at a time, with
    the energy and the Gauss-Radau factor of every iterate (as cg_energy)."""

    def __init__(self, apply_C, b, e0, normE, mu):
        self.C, self.x, self.r = apply_C, np.zeros_like(b), b.copy()
        self.p = self.r.copy()
        self.gam = inner(self.r, self.r)
        self.mu, self.normE = mu, normE
        self.phi = 1.0 / mu if mu > 0 else np.inf
        self.alpha_prev = self.gam_prev = None
        self.energy = [e0]            # energy of iterate i
        self.radau = []               # Gauss-Radau bound of iterate i (filled by the test of iterate i)
        self.i = 0
        self.done = False
        self.status = "maxit"

    def radau_bound(self):
        if self.i > 0 and self.mu > 0:
            t = self.phi - self.alpha_prev
            ph = t / (self.mu * t + self.gam / self.gam_prev)
            self.phi = ph if (t > 0 and 0 < ph < 1.0 / self.mu) else 1.0 / self.mu
        self.radau.append(self.gam * self.phi)
        return self.radau[-1]

    def step(self):
        q = self.C(self.p)
        pq = inner(self.p, q)
        if pq <= 0.0:
            raise FloatingPointError("operator not positive definite on the subspace")
        alpha = self.gam / pq
        self.x = self.x + alpha * self.p
        self.r = self.r - alpha * q
        gam_new = inner(self.r, self.r)
        self.energy.append(self.energy[-1] - alpha * self.gam)
        self.p = self.r + (gam_new / self.gam) * self.p
        self.alpha_prev, self.gam_prev, self.gam = alpha, self.gam, gam_new
        self.i += 1


def cg_pair_gap(primal, dual, normE, tol=1e-8, theta=0.01, chunk=8, maxit=20000):
    """The gap rule (module docstring) for one load E: primal = (apply_C, b, e0, mu)
    of the primal problem, dual = the same for the dual problem with J = E.
    Both CGs run iteration by iteration in lockstep; at iteration i (chunk
    c = i // chunk) a side reads the other's energy and Gauss-Radau bound at
    iterate min(c chunk - 1, its stop) for c >= 1 (its start energy and an
    infinite bound for c = 0).  Returns (primal run, dual run, the lower bounds
    on D* that the two stops used)."""
    runs = [_CGRun(*primal[:3], normE, primal[3]), _CGRun(*dual[:3], normE, dual[3])]
    n4 = normE ** 4
    dlow = [None, None]

    def upper_and_bound(i_energy, i_radau):
        return i_energy, i_radau                       # U and R of a primal iterate

    def lower_and_bound(V, RV):
        # L = |E|^4 / V and the bound R' on L* - L from the dual remainder RV
        return n4 / V, (n4 * RV / (V * (V - RV)) if V - RV > 0 else np.inf)

    def partner_state(k, i):
        o = runs[1 - k]
        c = i // chunk
        if c == 0:
            return o.energy[0], np.inf
        j = min(c * chunk - 1, o.i)
        return o.energy[j], o.radau[j]

    i = 0
    while not (runs[0].done and runs[1].done):
        for k, rk in enumerate(runs):
            if rk.done:
                continue
            R = rk.radau_bound()
            oe, orad = partner_state(k, i)
            if k == 0:
                U, RU = rk.energy[-1], R
                L, RL = lower_and_bound(oe, orad)
                own = RU
            else:
                U, RU = oe, orad
                L, RL = lower_and_bound(rk.energy[-1], R)
                own = RL
            d_low = (U - RU) - (L + RL)               # guaranteed: D* >= d_low
            if np.sqrt(rk.gam) <= tol * normE:
                rk.done, rk.status, dlow[k] = True, "residual", d_low
            elif d_low > 0 and own <= theta * d_low:
                rk.done, rk.status, dlow[k] = True, "gap", d_low
            elif i >= maxit:
                rk.done, dlow[k] = True, d_low
        for rk in runs:
            if not rk.done:
                rk.step()
        i += 1
    return runs[0], runs[1], dlow


def solve_pair_gap(prob, E, tol=1e-8, theta=0.01, chunk=8, mu=None, maxit=20000):
    """cg_pair_gap on the primal and dual Galerkin problems of a load E; mu: a
    pair (primal, dual) of spectrum lower bounds (default from the coefficients)."""
    E = np.asarray(E, float)
    sides = []
    for k, dual in enumerate((False, True)):
        C, coef = operator(prob, dual)
        m = spectrum_lower_bound(coef) if mu is None else mu[k]
        sides.append((C, -C(constant_field(E, prob.N)), zero_field_energy(prob, E, dual), m))
    return cg_pair_gap(sides[0], sides[1], float(np.linalg.norm(E)), tol, theta, chunk, maxit)

