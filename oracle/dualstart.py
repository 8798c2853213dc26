"""Dual start from the primal minimisers (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this package.

Proposition FD_odd_problem (ii), eq. FD_superposition_odd_A: on odd grids the
dual GaNi minimisers follow from the primal ones,

    e_b + j^(b) = A_N sum_a E_a (e_a + e^(a)),    E = A_{H,N}^{-1} e_b.

The remark on avoiding the dual solution applies the same formula to
approximate primal minimisers and restores conformity with the projection
onto J_N before further CG steps on the dual problem.  For the Galerkin scheme
with exact integration the superposition, taken with the exact product
P_N F_M (A_M F_M^{-1} pad) and the upper bound Abar in place of A_{H,N}, is an
admissible dual start (any field of J_N is).

Pinned by tests/test_oracle_dualstart.py: on odd grids the GaNi start from
converged primal minimisers is the dual GaNi minimiser (Proposition
FD_odd_problem (ii)) and needs no projection; the Ga start lies in J_N, its
energy bounds the converged dual energy from above and CG from it reaches the
same bounds.
"""
from __future__ import annotations

import numpy as np

from .galerkin import constant_field, ga_apply
from .spectral import apply_blockdiag, dft_nd, idft_nd, proj_J


def gani_dual_start(AN, Y, primal, A_HN, project=True):
    """GaNi: dual fluctuations j^(b) (grid values on the N grid) from the primal
    fluctuations e^(a) (grid values, list of d arrays (d, *N)) and A_{H,N}."""
    d = AN.shape[0]
    N = AN.shape[2:]
    I = np.eye(d)
    Einv = np.linalg.inv(A_HN)
    G = proj_J(N, np.asarray(Y, float))
    out = []
    for b in range(d):
        E = Einv[:, b]
        v = sum(E[a] * (primal[a] + I[a].reshape((d,) + (1,) * d)) for a in range(d))
        w = np.einsum("ij...,j...->i...", AN, v)                   # e_b + j^(b) on the grid
        if project:
            out.append(idft_nd(apply_blockdiag(G, dft_nd(w, d)), d).real)
        else:
            out.append(w - I[b].reshape((d,) + (1,) * d))
    return out


def ga_dual_start(prob, primal_hat, Abar):
    """Ga: dual fluctuations (Fourier coefficients on Z_N, full vectors) from the
    primal ones with the exact product on the doubled grid, projected onto J_N."""
    d = prob.d
    I = np.eye(d)
    Einv = np.linalg.inv(np.asarray(Abar, float))
    G = proj_J(prob.N, prob.Y)
    out = []
    for b in range(d):
        E = Einv[:, b]
        v = sum(E[a] * (constant_field(I[a], prob.N) + primal_hat[a]) for a in range(d))
        out.append(apply_blockdiag(G, ga_apply(prob.Atil, v, prob.N)))
    return out
