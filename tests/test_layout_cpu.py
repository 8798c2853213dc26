"""Host-side layout helpers of the binding (field vector <-> full spectrum),
checked on oracle solutions: fields in E_N / J_N survive the round trip and
the stored half determines the rest by Hermitian symmetry."""
import numpy as np
import pytest

import homgen
from oracle import galerkin as ga
from layout import spectrum_from_field, field_from_spectrum, basis_np


@pytest.mark.parametrize("cell,N", [
    (homgen.square_inclusion_cell(rho_in=5.0), (9, 7)),
    (homgen.pixel_cell(seed=3, P=5, values=(1.0, 9.0)), (7, 7)),
    (homgen.sphere_cell(seed=2, n=3, anisotropic=True), (5, 7, 5)),
])
@pytest.mark.parametrize("dual", [False, True])
def test_roundtrip_on_oracle_solutions(cell, N, dual):
    prob = ga.make_problem(cell, N)
    d = cell.d
    for a in range(d):
        x = ga.solve(prob, np.eye(d)[a], dual=dual, tol=1e-12).x
        c = field_from_spectrum(x, d, N, cell.Y, dual)
        back = spectrum_from_field(c, d, N, cell.Y, dual)
        assert np.abs(back - x).max() < 1e-12 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("d,N,Y", [(2, (5, 7), (1.0, 2.0)), (3, (5, 3, 7), (1.0, 0.5, 2.0))])
@pytest.mark.parametrize("dual", [False, True])
def test_basis_orthonormal_and_in_range_of_projection(d, N, Y, dual):
    T = basis_np(d, N, np.array(Y), dual)     # (m, d, ...)
    m = T.shape[0]
    G = np.einsum("ma...,mb...->ab...", T, T)
    H0 = (N[0] + 1) // 2
    from oracle.spectral import proj_E, proj_J
    P = (proj_J if dual else proj_E)(N, np.array(Y))[:, :, :H0]
    assert np.abs(G - P).max() < 1e-14
    gram = np.einsum("ma...,na...->mn...", T, T)
    nz = np.any(T != 0, axis=(0, 1))
    for i in range(m):
        for j in range(m):
            np.testing.assert_allclose(gram[i, j][nz], 1.0 if i == j else 0.0, atol=1e-14)
