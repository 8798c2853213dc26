"""Test-side adapters between the oracle's full Fourier spectra and the
library's field layout (include/hom.h): potential coefficients c(k) = T(k)^T
x_hat(k) on the stored half k_0 >= 0, with T(k) the orthonormal basis of the
range of G^E(k) (primal) or G^J(k) (dual), Def. of the projections (Sec. 2.3).

These live with the tests: they convert the oracle's output for comparison
with the GPU path and are never imported by the library or its binding.
"""
from __future__ import annotations

import numpy as np


def _freqs(n):
    return np.rint(np.fft.fftfreq(n, 1.0 / n)).astype(np.int64)


def basis_np(d, N, Y, dual):
    """T(k) of the field layout (include/hom.h) on the stored half, as an
    array (m, d, H0, N1[, N2]); zero at k = 0."""
    H0 = (N[0] + 1) // 2
    axes = [np.arange(H0)] + [_freqs(n) for n in N[1:d]]
    ks = np.meshgrid(*axes, indexing="ij")
    xi = np.stack([k / Y[a] for a, k in enumerate(ks)])
    nrm = np.sqrt(np.sum(xi * xi, axis=0))
    safe = np.where(nrm == 0, 1.0, nrm)
    n = xi / safe
    n[:, nrm == 0] = 0.0
    if not dual:
        return n[None]
    if d == 2:
        return np.stack([np.stack([-n[1], n[0]])])
    a = np.argmin(np.abs(n), axis=0)
    t1 = -np.take_along_axis(n, a[None], 0) * n
    for ax in range(3):
        t1[ax] += (a == ax)
    t1 /= np.where(np.linalg.norm(t1, axis=0) == 0, 1, np.linalg.norm(t1, axis=0))
    t2 = np.cross(n, t1, axis=0)
    T = np.stack([t1, t2])
    T[:, :, nrm == 0] = 0.0
    return T


def spectrum_from_field(c, d, N, Y, dual):
    """Full Fourier coefficients x_hat (d, *N) in FFT order from a field vector
    in the library layout (numpy, host)."""
    c = np.asarray(c)
    m = 1 if not dual else d - 1
    H0 = (N[0] + 1) // 2
    c = c.reshape((m, H0) + tuple(N[1:d]))
    T = basis_np(d, N, Y, dual)
    half = np.einsum("mg...,m...->g...", T, c)
    full = np.zeros((d,) + tuple(N), dtype=np.complex128)
    full[:, :H0] = half
    # k0 < 0 from x_hat(-k) = conj(x_hat(k))
    for i0 in range(H0, N[0]):
        src = N[0] - i0
        sl = half[:, src]
        idx = [np.mod(-_freqs(n), n) for n in N[1:d]]
        full[:, i0] = np.conj(sl[(slice(None),) + np.ix_(*idx)]) if idx else np.conj(sl)
    return full


def field_from_spectrum(xhat, d, N, Y, dual):
    """Library layout from full Fourier coefficients (d, *N): c = T^T x_hat on the stored half."""
    H0 = (N[0] + 1) // 2
    T = basis_np(d, N, Y, dual)
    half = np.asarray(xhat)[:, :H0]
    return np.einsum("mg...,g...->m...", T, half).reshape(-1)
