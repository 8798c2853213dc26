"""GaNi on general (odd or even) grids: Nyquist-aware projections (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this package.

Sec. 4.4 (Def. of the fully discrete projections for general grids) and
Sec. 5.2 (duality for general grids).  On a grid N the index set is
Z_N = {k : -N_a/2 <= k_a < N_a/2} (eq. index_sets); for even N_a it contains
the Nyquist frequencies k_a = -N_a/2, which the reduced set Z_N^r omits.  The
projections take the continuous Fourier symbols G^E(k), G^J(k) on Z_N^r and,
at the Nyquist frequencies, either 0 (G_{N,0}) or the identity (G_{N,I}):

    E_N = G^E_{N,0}[X_N],  J_N = G^J_{N,0}[X_N],
    E_N^app = G^E_{N,I}[X_N],  J_N^app = G^J_{N,I}[X_N].

GaNi (eq. FD_GaNi): A_{H,N} minimises the trapezoidal-rule energy with the
point values A(x_N^k) over E_N, B_{H,N} the one of A^-1 over J_N; the tilde
problems (eq. FD_GaNi_tilde) minimise over E_N^app and J_N^app.  Proposition
FD_even_problem: A_{H,N} = Btilde^-1, B_{H,N}^-1 = Atilde, and
B_{H,N}^-1 <= A_{H,N} (a duality gap on even grids).  The minimisers of E_N
and J_N have no Nyquist content, so they are trigonometric polynomials of
Z_N^r (for even N that is Z_{N-1}); step (iii) integrates them exactly with
the Ga quadrature of galerkin.py on the odd set.

Pinned by tests/test_oracle_even.py: the projections (identities of Lemma
matrix_orthogonality_E), Proposition FD_even_problem (i) and (iii), odd grids
against oracle/gani.py, homogeneous media, and the bound values the paper gives
for its open square at contrast 1e3 on the grid 1024.
"""
from __future__ import annotations

import numpy as np

from .galerkin import energy_matrix, make_problem
from . import spectral as sp


def freqs_general(L):
    """Integers of Z_L in FFT order: 0, 1, ..., then -floor(L/2), ..., -1."""
    return np.rint(np.fft.fftfreq(L, d=1.0 / L)).astype(np.int64)


def nyquist_mask(shape):
    """True at the frequencies with some k_a = -N_a / 2 (even N_a only)."""
    ks = np.meshgrid(*[freqs_general(L) for L in shape], indexing="ij")
    m = np.zeros(tuple(shape), dtype=bool)
    for L, k in zip(shape, ks):
        if L % 2 == 0:
            m |= k == -L // 2
    return m


def projections(shape, Y):
    """G^E_{N,0}, G^E_{N,I}, G^J_{N,0}, G^J_{N,I} as (d, d, *shape) arrays."""
    d = len(shape)
    ks = np.meshgrid(*[freqs_general(L) for L in shape], indexing="ij")
    xi = np.stack([k / Y[a] for a, k in enumerate(ks)])
    nrm2 = np.sum(xi * xi, axis=0)
    GE = xi[:, None] * xi[None, :] / np.where(nrm2 == 0.0, 1.0, nrm2)
    I = np.eye(d).reshape((d, d) + (1,) * d) * np.ones(tuple(shape))
    GJ = I - GE
    zero = (slice(None), slice(None)) + (0,) * d
    GE[zero] = 0.0
    GJ[zero] = 0.0
    nyq = nyquist_mask(shape)
    GE0, GJ0, GEI, GJI = GE.copy(), GJ.copy(), GE.copy(), GJ.copy()
    GE0[:, :, nyq] = 0.0
    GJ0[:, :, nyq] = 0.0
    GEI[:, :, nyq] = np.eye(d)[:, :, None]
    GJI[:, :, nyq] = np.eye(d)[:, :, None]
    return GE0, GEI, GJ0, GJI


def point_values(cell, shape, inverse=False, closed=False):
    """A(x_N^k), x^k = Y k / N for k in Z_N (any N): boxes |x_a - c_a| < h_a/2
    (<= with closed = True), balls |x - c| < R, periodic minimum image; pixels
    by the pixel containing the point."""
    d = cell.d
    Y = np.asarray(cell.Y, float)
    ks = np.meshgrid(*[freqs_general(L) for L in shape], indexing="ij")
    x = [Y[a] * ks[a] / shape[a] for a in range(d)]
    inv = lambda A: np.linalg.inv(np.asarray(A, float))
    if hasattr(cell, "phase"):
        P = cell.phase.shape
        vals = np.stack([inv(A) if inverse else np.asarray(A, float) for A in cell.phase_A])
        idx = [np.clip(np.floor((x[a] / Y[a] + 0.5) * P[a]).astype(np.int64), 0, P[a] - 1) for a in range(d)]
        return np.ascontiguousarray(np.moveaxis(vals[cell.phase[tuple(idx)]], (-2, -1), (0, 1)))
    A0 = inv(cell.A0) if inverse else np.asarray(cell.A0, float)
    out = np.broadcast_to(A0.reshape((d, d) + (1,) * d), (d, d) + tuple(shape)).copy()
    for kind, c, s, Ain in zip(cell.kind, cell.center, cell.size, cell.A):
        dl = [x[a] - c[a] for a in range(d)]
        dl = [v - Y[a] * np.round(v / Y[a]) for a, v in enumerate(dl)]
        if kind == "rect":
            inside = np.ones(tuple(shape), dtype=bool)
            for a in range(d):
                inside &= (np.abs(dl[a]) <= 0.5 * s[a]) if closed else (np.abs(dl[a]) < 0.5 * s[a])
        else:
            inside = sum(v * v for v in dl) < float(s[0]) ** 2
        out[:, :, inside] = (inv(Ain) if inverse else np.asarray(Ain, float))[:, :, None]
    return out


def _mean_inner(u, v):
    return float(np.mean(np.sum(u * v, axis=0)))


def _cg(coef, G, E, tol, maxit):
    """CG on the real-space system G (coef (E + x)) = 0, x in range(G), x0 = 0
    (eqs. linear_system_primal/dual with the projection G)."""
    d = coef.shape[0]
    shape = coef.shape[2:]

    def C(v):
        y = np.einsum("ab...,b...->a...", coef, v)
        return sp.idft_nd(sp.apply_blockdiag(G, sp.dft_nd(y, d)), d).real

    Ef = np.broadcast_to(np.asarray(E, float).reshape((d,) + (1,) * d), (d,) + tuple(shape)).copy()
    b = -C(Ef)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _mean_inner(r, r)
    it = 0
    while np.sqrt(rr) > tol * np.linalg.norm(E) and it < maxit:
        q = C(p)
        a = rr / _mean_inner(p, q)
        x = x + a * p
        r = r - a * q
        rn = _mean_inner(r, r)
        p = r + (rn / rr) * p
        rr = rn
        it += 1
    return x, it


def _energy(coef, fields):
    d = coef.shape[0]
    I = np.eye(d)
    out = np.zeros((d, d))
    for a in range(d):
        va = fields[a] + I[a].reshape((d,) + (1,) * d)
        Av = np.einsum("ij...,j...->i...", coef, va)
        for b in range(d):
            vb = fields[b] + I[b].reshape((d,) + (1,) * d)
            out[a, b] = _mean_inner(vb, Av)
    return out


def gani_general(cell, N, tol=1e-11, maxit=20000, closed=False, tilde=True):
    """GaNi on the grid N (odd or even): A_{H,N}, B_{H,N}, the tilde matrices of
    eq. FD_GaNi_tilde (tilde = True), and the exact bounds of the minimisers."""
    N = tuple(int(n) for n in (N if np.iterable(N) else [N] * cell.d))
    d = cell.d
    Y = np.asarray(cell.Y, float)
    AN = point_values(cell, N, closed=closed)
    BN = np.moveaxis(np.linalg.inv(np.moveaxis(AN, (0, 1), (-2, -1))), (-2, -1), (0, 1))
    GE0, GEI, GJ0, GJI = projections(N, Y)
    I = np.eye(d)
    xs, js, its = [], [], []
    for a in range(d):
        x, i1 = _cg(AN, GE0, I[a], tol, maxit)
        j, i2 = _cg(BN, GJ0, I[a], tol, maxit)
        xs.append(x)
        js.append(j)
        its.append((i1, i2))
    out = dict(A_HN=_energy(AN, xs), B_HN=_energy(BN, js), iters=its)
    if tilde:
        out["A_tilde"] = _energy(AN, [_cg(AN, GEI, I[a], tol, maxit)[0] for a in range(d)])
        out["B_tilde"] = _energy(BN, [_cg(BN, GJI, I[a], tol, maxit)[0] for a in range(d)])
    # step (iii): the minimisers are trigonometric polynomials of Z_N^r
    Nr = tuple(n if n % 2 else n - 1 for n in N)
    prob = make_problem(cell, Nr)

    def reduced(f):
        fh = sp.dft_nd(f, d)
        idx = tuple(np.mod(freqs_general(r), n) for r, n in zip(Nr, N))
        return fh[(slice(None),) + np.ix_(*idx)]

    A_up = energy_matrix(prob.Atil, [reduced(x) for x in xs], list(I))
    B_up = energy_matrix(prob.Btil, [reduced(j) for j in js], list(I))
    A_low = np.linalg.inv(B_up)
    out.update(A_up=A_up, B_up=B_up, A_low=A_low, D=0.5 * (A_up - A_low), fields_primal=xs, fields_dual=js)
    return out
