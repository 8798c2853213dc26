"""Galerkin approximation with numerical integration (GaNi): the paper's Algorithm.

Oracle (FP64).  Sec. 5 and Sec. 7: the bilinear forms are replaced by the
trapezoidal rule on the N grid, so the fully discrete coefficient is the
block-diagonal matrix of point values A_N = diag(A(x_N^k)) (eq. FD_A_GaNi)
and its inverse B_N = A_N^{-1}.  The systems (eqs. linear_system_primal/dual)

    F_N^{-1} G^E F_N A_N x = -F_N^{-1} G^E F_N A_N E,
    F_N^{-1} G^J F_N A_N^{-1} x = -F_N^{-1} G^J F_N A_N^{-1} J,

are solved by CG with x0 = 0, the inner product being the grid mean (the
isometry I_N of the Lemma on operators).  Step (iii) of the Algorithm then
evaluates the guaranteed bounds of the GaNi minimisers exactly, by the
double-grid quadrature (galerkin.energy_matrix).
"""
from __future__ import annotations

import numpy as np

from .spectral import proj_E, proj_J, apply_blockdiag, dft_nd, idft_nd
from .coefficients import point_values
from .galerkin import energy_matrix, make_problem


def _mean_inner(u, v):
    return float(np.mean(np.sum(u * v, axis=0)))


def gani_solve(AN, N, Y, E, dual=False, tol=1e-11, maxit=20000):
    d = len(N)
    G = proj_J(N, Y) if dual else proj_E(N, Y)
    coef = np.linalg.inv(np.moveaxis(AN, (0, 1), (-2, -1)))
    coef = np.moveaxis(coef, (-2, -1), (0, 1)) if dual else AN

    def C(x):
        y = np.einsum("ab...,b...->a...", coef, x)
        return idft_nd(apply_blockdiag(G, dft_nd(y, d)), d).real

    E = np.asarray(E, float)
    Ef = np.broadcast_to(E.reshape((d,) + (1,) * d), (d,) + tuple(N)).copy()
    b = -C(Ef)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _mean_inner(r, r)
    it = 0
    normE = float(np.linalg.norm(E))
    while np.sqrt(rr) > tol * normE and it < maxit:
        q = C(p)
        alpha = rr / _mean_inner(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = _mean_inner(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, coef


def gani_bounds(cell, N, tol=1e-11, maxit=20000):
    """The paper's Algorithm: GaNi matrices A_{H,N}, B_{H,N} and the guaranteed
    bounds of the GaNi minimisers (Def. GaNi, eq. GaNi_bounds)."""
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * cell.d))
    d = cell.d
    Y = np.asarray(cell.Y, float)
    AN = point_values(cell, N)
    I = np.eye(d)
    xs, js, its = [], [], []
    for a in range(d):
        x, it1, _ = gani_solve(AN, N, Y, I[a], dual=False, tol=tol, maxit=maxit)
        j, it2, BN = gani_solve(AN, N, Y, I[a], dual=True, tol=tol, maxit=maxit)
        xs.append(x)
        js.append(j)
        its.append((it1, it2))

    def disc_energy(coef, fields):
        out = np.zeros((d, d))
        for a in range(d):
            va = fields[a] + I[a].reshape((d,) + (1,) * d)
            Av = np.einsum("ij...,j...->i...", coef, va)
            for b in range(d):
                vb = fields[b] + I[b].reshape((d,) + (1,) * d)
                out[a, b] = _mean_inner(vb, Av)
        return out

    BN = np.moveaxis(np.linalg.inv(np.moveaxis(AN, (0, 1), (-2, -1))), (-2, -1), (0, 1))
    A_HN = disc_energy(AN, xs)
    B_HN = disc_energy(BN, js)
    prob = make_problem(cell, N)
    xh = [dft_nd(x, d) for x in xs]
    jh = [dft_nd(j, d) for j in js]
    A_up = energy_matrix(prob.Atil, xh, list(I))
    B_up = energy_matrix(prob.Btil, jh, list(I))
    A_low = np.linalg.inv(B_up)
    return dict(A_HN=A_HN, B_HN=B_HN, A_up=A_up, B_up=B_up, A_low=A_low,
                A_mean=0.5 * (A_up + A_low), D=0.5 * (A_up - A_low), iters=its)
