"""Dense Fourier-Galerkin system (Lemma Ga_full), for tiny grids.

Oracle (FP64).  Independent of FFTs and of the doubled grid: the bilinear form
of two trigonometric polynomials is

    a(u, v) = sum_{l, k in Z_N} v_hat(l)^H A_hat(l - k) u_hat(k),

(Lemma Ga_full, with (A_full)^{lk} = |Y|^{-1} int A phi_k phi_{-l} = A_hat(l - k)).
The unknown field lives in E_N (primal) or J_N (dual); at each k != 0 it is
expanded in an orthonormal basis T(k) of the range of G^E(k) (the unit vector
xi/|xi|) or of G^J(k) (its orthogonal complement).  The Galerkin equations for
the minimiser of a(E + x, E + x) (Def. homog_problem restricted to E_N) are

    sum_k T(l)^T A_hat(l - k) T(k) c(k) = -T(l)^T A_hat(l) E,   l in Z_N \\ {0},

solved directly.  A_hat comes from the closed-form coefficients, never from
the doubled-grid values.
"""
from __future__ import annotations

import itertools
import numpy as np


def _basis(k, Y, dual):
    xi = np.asarray(k, float) / np.asarray(Y, float)
    n = xi / np.linalg.norm(xi)
    if not dual:
        return n.reshape(-1, 1)
    # orthonormal complement of n
    d = len(n)
    Q, _ = np.linalg.qr(np.column_stack([n, np.eye(d)]))
    return Q[:, 1:d]


def _index_set(N):
    return [np.array(k) for k in itertools.product(*[range(-(n - 1) // 2, (n - 1) // 2 + 1) for n in N])]


def dense_matrix(Ahat_fn, N, Y, dual=False):
    """The Hermitian Galerkin matrix K of the system below (unknowns c(k) in
    the bases T(k), k in Z_N without 0), with the frequencies and bases."""
    ks = [k for k in _index_set(N) if np.any(k != 0)]
    bases = [_basis(k, Y, dual) for k in ks]
    m = bases[0].shape[1]
    n = len(ks) * m
    K = np.zeros((n, n), dtype=np.complex128)
    for i, (l, Tl) in enumerate(zip(ks, bases)):
        for j, (k, Tk) in enumerate(zip(ks, bases)):
            K[i * m:(i + 1) * m, j * m:(j + 1) * m] = Tl.T @ Ahat_fn(l - k) @ Tk
    return K, ks, bases


def dense_solve(Ahat_fn, N, Y, E, dual=False):
    """Solve the dense Galerkin system.

    Ahat_fn(n) -> d x d complex matrix A_hat(n) for an integer vector n
    (the series of A, or of A^{-1} for the dual).  Returns the Fourier
    coefficients of the minimiser as a dict {tuple(k): vector}."""
    K, ks, bases = dense_matrix(Ahat_fn, N, Y, dual)
    m = bases[0].shape[1]
    f = np.zeros(K.shape[0], dtype=np.complex128)
    E = np.asarray(E, float)
    for i, (l, Tl) in enumerate(zip(ks, bases)):
        f[i * m:(i + 1) * m] = -Tl.T @ (Ahat_fn(l) @ E)
    c = np.linalg.solve(K, f)
    return {tuple(k): Tk @ c[i * m:(i + 1) * m] for i, (k, Tk) in enumerate(zip(ks, bases))}


def dense_energy(Ahat_fn, N, fields, loads):
    """Energy matrix sum_{l,k} v_b(l)^H A_hat(l - k) v_a(k), v = E delta_0 + x_hat."""
    ks = _index_set(N)
    d = len(loads[0])
    vs = []
    for x, E in zip(fields, loads):
        v = {}
        for k in ks:
            v[tuple(k)] = np.array(x.get(tuple(k), np.zeros(d)), dtype=np.complex128)
        v[(0,) * len(N)] = v[(0,) * len(N)] + np.asarray(E, float)
        vs.append(v)
    n = len(fields)
    out = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            s = 0.0 + 0.0j
            for l in ks:
                vl = np.conj(vs[b][tuple(l)])
                for k in ks:
                    s += vl @ (Ahat_fn(l - k) @ vs[a][tuple(k)])
            out[a, b] = s.real
    return out


def dense_bounds(Ahat_fn, Bhat_fn, N, Y):
    d = len(N)
    I = np.eye(d)
    prim = [dense_solve(Ahat_fn, N, Y, I[a], dual=False) for a in range(d)]
    dual = [dense_solve(Bhat_fn, N, Y, I[a], dual=True) for a in range(d)]
    A_up = dense_energy(Ahat_fn, N, prim, list(I))
    B_up = dense_energy(Bhat_fn, N, dual, list(I))
    return dict(A_up=A_up, B_up=B_up, A_low=np.linalg.inv(B_up), prim=prim, dual=dual)


def ahat_lookup(Ahat_M):
    """Wrap an array (d, d, *M) on Z_M (FFT order) as a function of integer n."""
    M = Ahat_M.shape[2:]

    def f(n):
        idx = tuple(int(n[a]) % M[a] for a in range(len(M)))
        return Ahat_M[(slice(None), slice(None)) + idx]
    return f


def to_array(field, N, d):
    """dict {k: vector} -> (d, *N) array in FFT order."""
    out = np.zeros((d,) + tuple(N), dtype=np.complex128)
    for k, v in field.items():
        idx = tuple(int(k[a]) % N[a] for a in range(len(N)))
        out[(slice(None),) + idx] = v
    return out
