"""Pins for oracle.coefficients: Fourier coefficients against quadrature of the
defining integral (eq. FT_def), pixel images against a direct sum over pixel
boxes, the doubled-grid values against the explicit double sum (eq. MBA_GA)."""
import numpy as np
import pytest
from scipy import integrate

import homgen
from oracle import coefficients as co
from oracle.spectral import freq_mesh


def _quad_1d(n, lo, hi, Y):
    re = integrate.quad(lambda x: np.cos(2 * np.pi * n * x / Y), lo, hi, limit=200)[0]
    im = integrate.quad(lambda x: -np.sin(2 * np.pi * n * x / Y), lo, hi, limit=200)[0]
    return (re + 1j * im) / Y


def test_shifted_box_coefficients_match_quadrature():
    # A box of sides h at centre c: |Y|^-1 int_box exp(-2 pi i n.x/Y) dx is separable.
    Y = np.array([1.0, 2.0])
    h = np.array([0.3, 0.7])
    c = np.array([0.21, -0.4])
    shape = (7, 9)
    nm = freq_mesh(shape)
    closed = co.rect_hat(nm, h, Y) * co.shift_phase(nm, c, Y)
    for idx in [(0, 0), (1, 0), (0, 2), (3, 4), (6, 8), (2, 7)]:
        n = [nm[0][idx], nm[1][idx]]
        q = np.prod([_quad_1d(n[a], c[a] - h[a] / 2, c[a] + h[a] / 2, Y[a]) for a in range(2)])
        assert abs(closed[idx] - q) < 1e-12, (idx, closed[idx], q)


def test_ball_coefficients_match_radial_quadrature():
    Y = np.ones(3)
    R = 0.13
    shape = (5, 5, 5)
    nm = freq_mesh(shape)
    closed = co.ball_hat(nm, R, Y)
    for idx in [(0, 0, 0), (1, 0, 0), (1, 2, 0), (2, 2, 2), (4, 1, 3)]:
        xi = np.sqrt(sum(nm[a][idx] ** 2 for a in range(3)))
        # |Y|^-1 int_{|x|<R} exp(-2 pi i xi.x) dx = int_0^R 4 pi r^2 sin(2 pi xi r)/(2 pi xi r) dr
        f = (lambda r: 4 * np.pi * r * r) if xi == 0 else \
            (lambda r: 4 * np.pi * r * r * np.sinc(2 * xi * r))
        q = integrate.quad(f, 0, R, epsabs=1e-15, epsrel=1e-13)[0]
        assert abs(closed[idx] - q) < 1e-13 * max(1.0, abs(q)) + 1e-15


def test_inclusion_series_hermitian_and_mean():
    cell = homgen.sphere_cell(11, n=6, anisotropic=True)
    M = (9, 9, 9)
    Ah = co.fourier_inclusions(cell, M)
    # A real => A_hat(-n) = conj(A_hat(n)); A symmetric => A_hat(n) symmetric
    r = np.mod(-np.arange(9), 9)
    neg = Ah[(slice(None), slice(None)) + np.ix_(r, r, r)]
    np.testing.assert_allclose(neg, np.conj(Ah), atol=1e-15)
    np.testing.assert_allclose(Ah, np.swapaxes(Ah, 0, 1), atol=1e-15)
    # mean = A0 (1 - f) + sum A_in f_j
    vol = [4 / 3 * np.pi * s[0] ** 3 for s in cell.size]
    mean = cell.A0 * (1 - sum(vol)) + sum(v * A for v, A in zip(vol, cell.A))
    np.testing.assert_allclose(Ah[:, :, 0, 0, 0].real, mean, atol=1e-14)
    # series of A^{-1}: mean of A^{-1}
    Bh = co.fourier_inclusions(cell, M, inverse=True)
    meanB = np.linalg.inv(cell.A0) * (1 - sum(vol)) + sum(v * np.linalg.inv(A) for v, A in zip(vol, cell.A))
    np.testing.assert_allclose(Bh[:, :, 0, 0, 0].real, meanB, atol=1e-14)


@pytest.mark.parametrize("d,P,M", [(2, (5, 3), (9, 7)), (3, (3, 3, 3), (5, 5, 5))])
def test_pixel_series_equals_sum_of_pixel_boxes(d, P, M):
    rng = np.random.default_rng(5)
    phase = rng.integers(0, 3, size=P).astype(np.int32)
    pA = np.stack([homgen.random_spd(rng, d) for _ in range(3)])
    pix = homgen.Pixels(d=d, Y=np.ones(d) * np.array([1.0, 1.5, 0.8][:d]), phase=phase, phase_A=pA)
    # direct: every pixel is a box inclusion in a zero matrix phase
    Y = pix.Y
    nm = freq_mesh(M)
    direct = np.zeros((d, d) + M, dtype=np.complex128)
    h = Y / np.array(P)
    for i in np.ndindex(*P):
        c = Y * (-0.5 + (np.array(i) + 0.5) / np.array(P))
        f = co.rect_hat(nm, h, Y) * co.shift_phase(nm, c, Y)
        direct += pA[phase[i]].reshape((d, d) + (1,) * d) * f[None, None]
    np.testing.assert_allclose(co.fourier_pixels(pix, M), direct, atol=1e-13)


@pytest.mark.parametrize("M", [(5, 7), (3, 5, 3)])
def test_double_grid_equals_explicit_sum(M):
    d = len(M)
    cell = homgen.Inclusions(d=d, Y=np.ones(d), A0=np.eye(d))
    cell.add("rect", np.full(d, 0.1), np.full(d, 0.4), 3.0 * np.eye(d) + 0.5)
    Ah = co.fourier_inclusions(cell, M)
    np.testing.assert_allclose(co.double_grid(Ah), co.double_grid_direct(Ah), atol=1e-12)


def test_double_grid_of_homogeneous_is_constant():
    A0 = np.array([[2.0, 0.3], [0.3, 1.0]])
    cell = homgen.homogeneous_cell(2, A0)
    At = co.double_grid(co.fourier_inclusions(cell, (9, 9)))
    np.testing.assert_allclose(At, np.broadcast_to(A0[:, :, None, None], At.shape), atol=1e-15)


def test_point_values_open_set_and_periodic_wrap():
    cell = homgen.Inclusions(d=2, Y=np.ones(2), A0=np.eye(2))
    cell.add("rect", np.array([0.45, 0.0]), np.array([0.3, 0.2]), 5 * np.eye(2))
    A = co.point_values(cell, (11, 11))
    # grid x = k/11; inclusion covers |x - 0.45| < 0.15 periodically, |y| < 0.1
    k = np.rint(np.fft.fftfreq(11, 1 / 11)).astype(int)
    for i in range(11):
        for j in range(11):
            x, y = k[i] / 11, k[j] / 11
            dx = x - 0.45
            dx -= np.round(dx)
            inside = abs(dx) < 0.15 and abs(y) < 0.1
            assert A[0, 0, i, j] == (5.0 if inside else 1.0)


def test_smoothing_filter_stencil_and_invariants():
    """Sec. 8.3 smoothing: a single inclusion pixel spreads as the stencil 1-2-1 x 1-2-1
    (weights 4, 2, 1 sixteenths); constants stay; mass is conserved; the filter commutes
    with transposition and with periodic shifts."""
    f = np.zeros((7, 9), dtype=np.int64)
    f[3, 4] = 1
    g = co.smooth_characteristic(f)
    expect = np.zeros_like(f)
    expect[2:5, 3:6] = [[1, 2, 1], [2, 4, 2], [1, 2, 1]]
    assert (g == expect).all()
    # periodic wrap at the corner
    f = np.zeros((5, 5), dtype=np.int64)
    f[0, 0] = 1
    g = co.smooth_characteristic(f)
    assert g[4, 4] == 1 and g[0, 4] == 2 and g[4, 0] == 2 and g[0, 0] == 4 and g.sum() == 16
    rng = np.random.default_rng(3)
    f = (rng.random((25, 15)) < 0.4).astype(np.int64)
    g = co.smooth_characteristic(f)
    assert (co.smooth_characteristic(np.ones_like(f)) == 16).all()
    assert g.sum() == 16 * f.sum() and g.min() >= 0 and g.max() <= 16
    assert (co.smooth_characteristic(f.T) == g.T).all()
    assert (co.smooth_characteristic(np.roll(f, (2, -3), axis=(0, 1))) == np.roll(g, (2, -3), axis=(0, 1))).all()
