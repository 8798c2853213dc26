"""Fourier coefficients of the material coefficient and its double-grid values.

Oracle (FP64).  Follows
  * eq. (FT_def): A_hat(n) = |Y|^{-1} int_Y A(x) phi_{-n}(x) dx;
  * Lemma "bounds_for_matrix-inclusion" / eq. (A_with_inclusions):
        A_hat(n) = A0 delta_{n0} + sum_j A_j f_hat_j(n) phi_{-n}(x_j),
    with A_j = (coefficient inside inclusion j) - A0 for indicator topologies;
  * Remark "inclusion": f_hat of a centred box,
        rect_hat(n) = |Y|^{-1} prod_a h_a sinc(h_a n_a / Y_a);
  * Lemma "integral_eval_double_grid", eq. (MBA_GA): the coefficient on the
    doubled grid, A_{2N-1}(x^k) = sum_{n in Z_{2N-1}} omega^{kn} A_hat(n).

The dual problem needs the Fourier series of A^{-1}.  For non-overlapping
indicator inclusions A^{-1} = A0^{-1} + sum_j f_j(x - x_j) (A_in,j^{-1} - A0^{-1}),
so the same formula applies with inverted phase matrices (reading R3).

Balls (3D) are not given in closed form in the paper (it defers to another
work); here f_hat(n) = |Y|^{-1} 4 pi (sin t - t cos t) / kappa^3 with
kappa = 2 pi |xi(n)|, t = kappa R, the textbook Fourier transform of a ball.

Pinned by tests/test_oracle_coefficients.py: quadrature of the defining
integral for rect and ball, pixel images against a direct sum over pixel boxes,
the double-grid values against the direct double sum, Hermitian symmetry.
"""
from __future__ import annotations

import numpy as np

from .spectral import freqs, freq_mesh, idft_nd

TWO_PI = 2.0 * np.pi


def rect_hat(n_mesh, h, Y):
    """Fourier coefficients of a centred box of side lengths h (Remark inclusion)."""
    out = np.ones(n_mesh[0].shape)
    for a, n in enumerate(n_mesh):
        out = out * (h[a] / Y[a]) * np.sinc(h[a] * n / Y[a])
    return out


def ball_hat(n_mesh, R, Y):
    """Fourier coefficients of a centred ball of radius R (3D, textbook form)."""
    xi2 = sum((n / Y[a]) ** 2 for a, n in enumerate(n_mesh))
    kappa = TWO_PI * np.sqrt(xi2)
    t = kappa * R
    vol = np.prod(Y)
    out = np.empty(kappa.shape)
    small = t < 1e-2
    # series of 4 pi (sin t - t cos t)/kappa^3 = (4/3) pi R^3 (1 - t^2/10 + t^4/280 - ...)
    ts = t[small]
    out[small] = (4.0 / 3.0) * np.pi * R ** 3 * (1.0 - ts ** 2 / 10.0 + ts ** 4 / 280.0)
    tb, kb = t[~small], kappa[~small]
    out[~small] = 4.0 * np.pi * (np.sin(tb) - tb * np.cos(tb)) / kb ** 3
    return out / vol


def shift_phase(n_mesh, x, Y):
    """phi_{-n}(x) = exp(-2 pi i sum_a n_a x_a / Y_a)."""
    ph = sum(n * (x[a] / Y[a]) for a, n in enumerate(n_mesh))
    return np.exp(-1j * TWO_PI * ph)


def _inv(A):
    return np.linalg.inv(A)


def fourier_inclusions(cell, shape, inverse=False):
    """A_hat(n) (or the series of A^{-1}) on the index set of `shape` (FFT order).

    Returns a complex array (d, d, *shape)."""
    d = cell.d
    Y = np.asarray(cell.Y, float)
    n_mesh = freq_mesh(shape)
    A0 = _inv(cell.A0) if inverse else np.asarray(cell.A0, float)
    out = np.zeros((d, d) + tuple(shape), dtype=np.complex128)
    out[(slice(None), slice(None)) + (0,) * d] = A0
    for kind, c, s, Ain in zip(cell.kind, cell.center, cell.size, cell.A):
        Aj = (_inv(Ain) if inverse else Ain) - A0
        if kind == "rect":
            f = rect_hat(n_mesh, s, Y)
        elif kind == "ball":
            assert d == 3, "ball inclusions are 3D"
            f = ball_hat(n_mesh, float(s[0]), Y)
        else:
            raise ValueError(kind)
        fs = f * shift_phase(n_mesh, c, Y)
        out += Aj.reshape((d, d) + (1,) * d) * fs[None, None]
    return out


def fourier_pixels(pix, shape, inverse=False):
    """Fourier coefficients of a pixel-wise constant coefficient on `shape`.

    Pixel i along axis a is the box of side Y_a/P_a centred at
    c_i = Y_a (-1/2 + (i + 1/2)/P_a).  Summing box coefficients (Remark
    inclusion) over all pixels gives
        A_hat(n) = prod_a [ sinc(n_a/P_a)/P_a * exp(-2 pi i n_a (1/(2P_a) - 1/2)) ]
                   * sum_i A_i exp(-2 pi i sum_a n_a i_a / P_a),
    and the last sum is a P-point DFT evaluated at n mod P.
    """
    d = pix.d
    P = pix.phase.shape
    vals = np.linalg.inv(pix.phase_A) if inverse else pix.phase_A
    img = vals[pix.phase]                     # (*P, d, d)
    img = np.moveaxis(img, (-2, -1), (0, 1))   # (d, d, *P)
    D = np.fft.fftn(img, axes=tuple(range(2, 2 + d)))
    n_mesh = freq_mesh(shape)
    idx = tuple(np.mod(n, Pa) for n, Pa in zip(n_mesh, P))
    out = D[(slice(None), slice(None)) + idx]
    fac = np.ones(n_mesh[0].shape, dtype=np.complex128)
    for a, n in enumerate(n_mesh):
        fac = fac * np.sinc(n / P[a]) / P[a] * np.exp(-1j * TWO_PI * n * (0.5 / P[a] - 0.5))
    return out * fac[None, None]


def fourier_coefficients(cell, shape, inverse=False):
    if hasattr(cell, "phase"):
        return fourier_pixels(cell, shape, inverse)
    return fourier_inclusions(cell, shape, inverse)


def double_grid(Ahat):
    """Coefficient on the doubled grid, eq. (MBA_GA):
    A_M(x^k) = sum_{n in Z_M} omega_M^{kn} A_hat(n)  (an unnormalised iDFT).

    Ahat: (d, d, *M) complex on Z_M in FFT order.  Returns the real part and
    checks that the imaginary part is at rounding level."""
    d = Ahat.shape[0]
    A = idft_nd(Ahat, d)
    scale = max(np.abs(A.real).max(), 1.0)
    assert np.abs(A.imag).max() <= 1e-11 * scale, "coefficient series is not Hermitian"
    return np.ascontiguousarray(A.real)


def double_grid_direct(Ahat):
    """Same as double_grid, by the explicit double sum (for small grids only)."""
    d = Ahat.shape[0]
    shape = Ahat.shape[2:]
    k_mesh = freq_mesh(shape)
    out = np.zeros(Ahat.shape, dtype=np.complex128)
    flat_n = [m.ravel() for m in k_mesh]
    Af = Ahat.reshape(d, d, -1)
    for pos in np.ndindex(*shape):
        ph = sum(k_mesh[a][pos] * flat_n[a] / shape[a] for a in range(len(shape)))
        w = np.exp(1j * TWO_PI * ph)
        out[(slice(None), slice(None)) + pos] = Af @ w
    return out.real


def point_values(cell, shape, inverse=False):
    """A(x_N^k) at the grid points x^k = (Y_a k_a / N_a)_a, k in Z_N (eq. grid_points).

    Used by the GaNi scheme (eq. FD_A_GaNi).  A point belongs to a box
    inclusion iff |x_a - c_a| < h_a/2 for all a (open set, as in eq. S), to a
    ball iff |x - c| < R, with periodic minimum-image distances."""
    d = cell.d
    Y = np.asarray(cell.Y, float)
    k_mesh = freq_mesh(shape)
    x = [Y[a] * k_mesh[a] / shape[a] for a in range(d)]
    if hasattr(cell, "phase"):
        P = cell.phase.shape
        vals = np.linalg.inv(cell.phase_A) if inverse else cell.phase_A
        idx = []
        for a in range(d):
            i = np.floor((x[a] / Y[a] + 0.5) * P[a]).astype(np.int64)
            idx.append(np.clip(i, 0, P[a] - 1))
        img = vals[cell.phase[tuple(idx)]]
        return np.ascontiguousarray(np.moveaxis(img, (-2, -1), (0, 1)))
    A0 = _inv(cell.A0) if inverse else np.asarray(cell.A0, float)
    out = np.broadcast_to(A0.reshape((d, d) + (1,) * d), (d, d) + tuple(shape)).copy()
    for kind, c, s, Ain in zip(cell.kind, cell.center, cell.size, cell.A):
        dl = [x[a] - c[a] for a in range(d)]
        dl = [v - Y[a] * np.round(v / Y[a]) for a, v in enumerate(dl)]
        if kind == "rect":
            inside = np.ones(shape, dtype=bool)
            for a in range(d):
                inside &= np.abs(dl[a]) < 0.5 * s[a]
        else:
            inside = sum(v * v for v in dl) < float(s[0]) ** 2
        val = _inv(Ain) if inverse else Ain
        out[:, :, inside] = val[:, :, None]
    return out


def smooth_characteristic(f):
    """The coefficient smoothing filter of the paper's fly-ash example (Sec. 8.3):
    every grid value of a 2D characteristic function is replaced by a local
    average, 4/16 of itself, 2/16 of each of its four axis neighbours and 1/16
    of each of its four diagonal neighbours (periodic).  Returns the integer
    image 16 f_smoothed (exact: the weights are sixteenths)."""
    f = np.asarray(f, dtype=np.int64)
    assert f.ndim == 2
    sh = lambda a, b: np.roll(np.roll(f, -a, axis=0), -b, axis=1)     # f at k + (a, b)
    return (4 * f
            + 2 * (sh(1, 0) + sh(-1, 0) + sh(0, 1) + sh(0, -1))
            + (sh(1, 1) + sh(-1, -1) + sh(-1, 1) + sh(1, -1)))


def z_half_M(N):
    """Shape of the doubled grid for an N grid: M = 2N - 1 per axis."""
    return tuple(2 * n - 1 for n in N)


__all__ = ["rect_hat", "ball_hat", "shift_phase", "fourier_inclusions", "fourier_pixels", "smooth_characteristic",
           "fourier_coefficients", "double_grid", "double_grid_direct", "point_values",
           "z_half_M", "freqs"]
