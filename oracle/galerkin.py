"""Galerkin scheme without numerical integration ("Ga"), CG and guaranteed bounds.

Oracle (FP64, full complex spectra, full d x d coefficients).

Discretisation (Sec. 6): trial/test fields are trigonometric polynomials of
T_N (odd N), stored by their Fourier coefficients on Z_N.  The bilinear form
a(u, v) = (A u, v)_{L2} is evaluated exactly by the double-grid quadrature
(Lemma integral_eval_double_grid), so the Galerkin operator on Fourier
coefficients is

    (K u_hat)(k) = P_N F_M [ A_M . F_M^{-1} pad_M(u_hat) ](k),   k in Z_N,

with M = 2N - 1, A_M the coefficient on the doubled grid (eq. MBA_GA) and
F_M, F_M^{-1} the DFT pair of eq. (DFT).  Equivalently (K u_hat)(k) =
sum_m A_hat(k - m) u_hat(m) (Lemma Ga_full), which tests/test_oracle_dense.py
checks against an independent dense assembly.

Linear systems (Sec. 7.1, eqs. linear_system_primal/dual, with the exact
form in place of the trapezoidal one):
    primal:  G^E K x = -G^E K E,   x in E_N      (coefficient A)
    dual:    G^J K' x = -G^J K' J, x in J_N      (coefficient series of A^{-1})
solved by Hestenes-Stiefel CG from x0 = 0 with the stopping rule of the
"Convergence criteria" remark: ||r_i|| <= eps ||E||, r = -G K (x_i + E), the
norm being the L2 norm (Parseval).

Bounds (Def. upper_lower_bounds, eq. GaNi_bounds):
    Abar_ab = a(e_b + x^(b), e_a + x^(a)),  Bbar_ab = a^{-1}(e_b + j^(b), e_a + j^(a)),
evaluated by the double-grid quadrature; lower bound Bbar^{-1}; mean and
guaranteed error D of eq. (approx_homog_with_error).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .spectral import pad, trunc, proj_E, proj_J, apply_blockdiag, inner, dft_nd, idft_nd
from .coefficients import fourier_coefficients, double_grid


@dataclass
class GaProblem:
    d: int
    N: tuple
    M: tuple
    Y: np.ndarray
    Ahat: np.ndarray     # (d, d, *M) Fourier coefficients of A on Z_M
    Bhat: np.ndarray     # same for A^{-1}
    Atil: np.ndarray     # (d, d, *M) real, A on the doubled grid
    Btil: np.ndarray


def make_problem(cell, N):
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * cell.d))
    assert all(n % 2 == 1 for n in N), "odd grids only"
    M = tuple(2 * n - 1 for n in N)
    Ahat = fourier_coefficients(cell, M, inverse=False)
    Bhat = fourier_coefficients(cell, M, inverse=True)
    return GaProblem(d=cell.d, N=N, M=M, Y=np.asarray(cell.Y, float), Ahat=Ahat, Bhat=Bhat,
                     Atil=double_grid(Ahat), Btil=double_grid(Bhat))


def to_grid(xhat, M):
    """Values on the doubled grid of the trigonometric polynomial with
    coefficients xhat on Z_N: F_M^{-1} pad_M(xhat) (real for Hermitian data)."""
    d = len(M)
    u = idft_nd(pad(xhat, M), d)
    return u.real


def ga_apply(coef_M, xhat, N):
    """K x_hat = P_N F_M [coef_M . F_M^{-1} pad_M x_hat]  (exact Galerkin product)."""
    d = len(N)
    M = coef_M.shape[2:]
    u = idft_nd(pad(xhat, M), d)                 # complex in general
    w = np.einsum("ab...,b...->a...", coef_M, u)
    return trunc(dft_nd(w, d), N)


def constant_field(E, N):
    """Fourier coefficients on Z_N of the constant field E (only k = 0)."""
    d = len(N)
    out = np.zeros((d,) + tuple(N), dtype=np.complex128)
    out[(slice(None),) + (0,) * d] = E
    return out


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    res_hist: list
    converged: bool


def cg(apply_C, b, x0, tol, normE, maxit=20000, callback=None):
    """Hestenes-Stiefel conjugate gradients for C x = b on the subspace that
    contains b and x0 (Sec. 7.1 Remark: the Krylov spaces stay in E_N/J_N)."""
    x = x0.copy()
    r = b - apply_C(x)
    p = r.copy()
    rr = inner(r, r)
    hist = [np.sqrt(rr)]
    it = 0
    while np.sqrt(rr) > tol * normE and it < maxit:
        q = apply_C(p)
        pq = inner(p, q)
        if pq <= 0.0:
            raise FloatingPointError("operator not positive definite on the subspace")
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = inner(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr))
        if callback is not None:
            callback(x)
    return CGResult(x=x, iters=it, res_hist=hist, converged=bool(np.sqrt(rr) <= tol * normE))


def solve(prob, E, dual=False, tol=1e-11, maxit=20000, x0=None, callback=None):
    """Minimiser of the primal (or dual) Galerkin problem for load E."""
    E = np.asarray(E, float)
    coef = prob.Btil if dual else prob.Atil
    G = proj_J(prob.N, prob.Y) if dual else proj_E(prob.N, prob.Y)

    def C(x):
        return apply_blockdiag(G, ga_apply(coef, x, prob.N))

    b = -C(constant_field(E, prob.N))
    if x0 is None:
        x0 = np.zeros_like(b)
    else:
        x0 = apply_blockdiag(G, x0)
    return cg(C, b, x0, tol, float(np.linalg.norm(E)), maxit, callback)


def energy_matrix(coef_M, fields, loads):
    """E_ab = mean over the doubled grid of v_b . coef v_a with
    v_a = loads[a] + (field a on the grid): the exact bilinear form
    (Lemma integral_eval_double_grid)."""
    n = len(fields)
    M = coef_M.shape[2:]
    vs = []
    for x, E in zip(fields, loads):
        v = to_grid(x, M)
        v = v + np.asarray(E, float).reshape((-1,) + (1,) * len(M))
        vs.append(v)
    out = np.zeros((n, n))
    for a in range(n):
        Av = np.einsum("ij...,j...->i...", coef_M, vs[a])
        for b in range(n):
            out[a, b] = float(np.mean(np.sum(vs[b] * Av, axis=0)))
    return out


def bounds_from_fields(prob, prim, dual):
    d = prob.d
    I = np.eye(d)
    A_up = energy_matrix(prob.Atil, prim, list(I))
    B_up = energy_matrix(prob.Btil, dual, list(I))
    A_low = np.linalg.inv(B_up)
    return dict(A_up=A_up, B_up=B_up, A_low=A_low,
                A_mean=0.5 * (A_up + A_low), D=0.5 * (A_up - A_low))


def bounds(prob, tol=1e-11, maxit=20000, x0_primal=None, x0_dual=None):
    """Full Ga procedure: d primal + d dual solves and the bounds."""
    d = prob.d
    I = np.eye(d)
    prim, dual, it_p, it_d = [], [], [], []
    for a in range(d):
        rp = solve(prob, I[a], dual=False, tol=tol, maxit=maxit,
                   x0=None if x0_primal is None else x0_primal[a])
        rd = solve(prob, I[a], dual=True, tol=tol, maxit=maxit,
                   x0=None if x0_dual is None else x0_dual[a])
        prim.append(rp.x)
        dual.append(rd.x)
        it_p.append(rp.iters)
        it_d.append(rd.iters)
    out = bounds_from_fields(prob, prim, dual)
    out.update(iters_primal=it_p, iters_dual=it_d, fields_primal=prim, fields_dual=dual)
    return out


def voigt_reuss(prob):
    """<A> = A_hat(0) (Voigt) and <A^{-1}>^{-1} (Reuss), Remark Aeff_spd."""
    d = prob.d
    z = (slice(None), slice(None)) + (0,) * d
    return prob.Ahat[z].real.copy(), np.linalg.inv(prob.Bhat[z].real)
