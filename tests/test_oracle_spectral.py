"""Pins for oracle.spectral: DFT conventions (eq. DFT, Lemma on phi_k at grid
points) against explicit sums, and the Helmholtz projections (Def.
projection, Lemma matrix_orthogonality)."""
import itertools

import numpy as np
import pytest

from oracle import spectral as sp


def test_freqs_odd():
    assert list(sp.freqs(5)) == [0, 1, 2, -2, -1]
    assert list(sp.freqs(1)) == [0]
    with pytest.raises(AssertionError):
        sp.freqs(4)


@pytest.mark.parametrize("shape", [(5,), (3, 5), (3, 3, 5)])
def test_dft_matches_explicit_sum(shape):
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d = len(shape)
    n = np.prod(shape)
    np.testing.assert_allclose(sp.dft_nd(u, d), sp.naive_dft(u, -1) / n, atol=1e-13)
    np.testing.assert_allclose(sp.idft_nd(u, d), sp.naive_dft(u, +1), atol=1e-12)


def test_idft_evaluates_trig_polynomial_at_grid_points():
    # u(x) = sum_k u_hat(k) exp(2 pi i k.x/Y) evaluated at x^m = Y m / N
    rng = np.random.default_rng(2)
    N = (5, 7)
    Y = np.array([1.0, 2.5])
    uh = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    vals = sp.idft_nd(uh, 2)
    f0, f1 = sp.freqs(N[0]), sp.freqs(N[1])
    for i, j in itertools.product(range(N[0]), range(N[1])):
        x = np.array([Y[0] * f0[i] / N[0], Y[1] * f1[j] / N[1]])
        s = sum(uh[a, b] * np.exp(2j * np.pi * (f0[a] * x[0] / Y[0] + f1[b] * x[1] / Y[1]))
                for a in range(N[0]) for b in range(N[1]))
        assert abs(s - vals[i, j]) < 1e-12


def test_pad_trunc_roundtrip_and_placement():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 5, 3)) + 0j
    y = sp.pad(x, (9, 5))
    np.testing.assert_array_equal(sp.trunc(y, (5, 3)), x)
    # frequency -2 of a length-5 axis sits at index 7 of a length-9 axis
    assert y[0, 7, 0] == x[0, 3, 0]
    assert np.count_nonzero(y) == x.size


@pytest.mark.parametrize("shape,Y", [((5, 7), (1.0, 1.0)), ((3, 5, 5), (1.0, 2.0, 0.5))])
def test_projections_resolution_of_identity_and_orthogonality(shape, Y):
    Y = np.array(Y)
    d = len(shape)
    GU, GE, GJ = sp.proj_U(shape), sp.proj_E(shape, Y), sp.proj_J(shape, Y)
    I = np.eye(d).reshape((d, d) + (1,) * d)
    np.testing.assert_allclose(GU + GE + GJ, np.broadcast_to(I, GE.shape), atol=1e-15)
    mm = lambda A, B: np.einsum("ab...,bc...->ac...", A, B)
    for G in (GU, GE, GJ):
        np.testing.assert_allclose(mm(G, G), G, atol=1e-14)                 # idempotent
        np.testing.assert_allclose(G, np.swapaxes(G, 0, 1), atol=1e-15)    # symmetric
    for A, B in ((GU, GE), (GU, GJ), (GE, GJ)):
        np.testing.assert_allclose(mm(A, B), 0.0, atol=1e-14)
    # G^E(k) xi(k) = xi(k): curl-free fields are gradients
    xi = sp.xi_mesh(shape, Y)
    np.testing.assert_allclose(sp.apply_blockdiag(GE, xi), xi, atol=1e-14)


def test_parseval_inner_product_equals_grid_mean():
    # (u, v)_{L2} = sum_k u_hat.conj(v_hat) = grid mean of u.v on the N grid (isometry I_N)
    rng = np.random.default_rng(4)
    N = (7, 5)
    u = rng.standard_normal((2,) + N)
    v = rng.standard_normal((2,) + N)
    uh, vh = sp.dft_nd(u, 2), sp.dft_nd(v, 2)
    assert abs(sp.inner(uh, vh) - np.mean(np.sum(u * v, axis=0))) < 1e-14
