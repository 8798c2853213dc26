"""Index sets, DFT conventions and Helmholtz projections (oracle, FP64).

Follows Sec. 2.2-2.3 (Fourier series, Def. of the projections G^U, G^E, G^J)
and Sec. 4.2 (index sets Z_N, grid points, DFT/iDFT matrices F_N, F_N^{-1}).

Array convention: an axis of odd length L stores frequency k (or grid index k)
at position k mod L ("FFT order"), so k in Z_L = {-(L-1)/2, ..., (L-1)/2}.

Pinned by tests/test_oracle_spectral.py (naive DFT sums, projection identities).
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import scipy.fft as sfft

# worker threads for the FFT library (pocketfft); the CPU baseline states this count
WORKERS = int(os.environ.get("HOM_ORACLE_WORKERS", os.cpu_count() or 1))


def freqs(L):
    """Integer frequencies of Z_L in FFT order (odd L)."""
    assert L % 2 == 1, "odd grids only"
    return np.rint(np.fft.fftfreq(L, d=1.0 / L)).astype(np.int64)


def freq_mesh(shape):
    """List of d integer arrays k_alpha over the grid of `shape` (FFT order)."""
    axes = [freqs(L) for L in shape]
    return np.meshgrid(*axes, indexing="ij")


def xi_mesh(shape, Y):
    """xi(k) = (k_alpha / Y_alpha)_alpha as an array (d, *shape)."""
    ks = freq_mesh(shape)
    return np.stack([k / Y[a] for a, k in enumerate(ks)])


def dft_nd(u, d):
    """F_N applied to the last d axes."""
    axes = tuple(range(u.ndim - d, u.ndim))
    n = np.prod([u.shape[a] for a in axes])
    return sfft.fftn(u, axes=axes, workers=WORKERS) / n


def idft_nd(uhat, d):
    """F_N^{-1} applied to the last d axes."""
    axes = tuple(range(uhat.ndim - d, uhat.ndim))
    n = np.prod([uhat.shape[a] for a in axes])
    return sfft.ifftn(uhat, axes=axes, workers=WORKERS) * n


def naive_dft(u, sign=-1):
    """Direct O(|N|^2) evaluation of sum_m omega^{sign*k*m} u(m) over all axes."""
    shape = u.shape
    out = np.zeros(shape, dtype=np.complex128)
    kk = [freqs(L) for L in shape]
    for kidx in itertools.product(*[range(L) for L in shape]):
        s = 0.0 + 0.0j
        for midx in itertools.product(*[range(L) for L in shape]):
            ph = sum(kk[a][kidx[a]] * kk[a][midx[a]] / shape[a] for a in range(len(shape)))
            s += np.exp(sign * 2j * np.pi * ph) * u[midx]
        out[kidx] = s
    return out


def pad(xhat, Mshape):
    """Embed Fourier coefficients on Z_N into Z_M (M >= N): zero elsewhere.

    xhat has shape (..., *Nshape); frequency k is placed at position k mod M.
    """
    d = len(Mshape)
    Nshape = xhat.shape[-d:]
    out = np.zeros(xhat.shape[:-d] + tuple(Mshape), dtype=np.complex128)
    idx = tuple(np.mod(freqs(N), M) for N, M in zip(Nshape, Mshape))
    out[(Ellipsis,) + np.ix_(*idx)] = xhat
    return out


def trunc(yhat, Nshape):
    """Truncation P_N: keep the Fourier coefficients with k in Z_N (Def. operators)."""
    d = len(Nshape)
    Mshape = yhat.shape[-d:]
    idx = tuple(np.mod(freqs(N), M) for N, M in zip(Nshape, Mshape))
    return yhat[(Ellipsis,) + np.ix_(*idx)]


def proj_E(shape, Y):
    """G^E(k) = xi xi^T / (xi . xi) for k != 0, 0 at k = 0 (Def. projection).

    Returns an array (d, d, *shape)."""
    xi = xi_mesh(shape, Y)
    nrm2 = np.sum(xi * xi, axis=0)
    safe = np.where(nrm2 == 0.0, 1.0, nrm2)
    G = xi[:, None] * xi[None, :] / safe
    G[(slice(None), slice(None)) + (0,) * len(shape)] = 0.0
    return G


def proj_J(shape, Y):
    """G^J(k) = I - G^E(k) for k != 0, 0 at k = 0 (Def. projection)."""
    d = len(shape)
    GE = proj_E(shape, Y)
    I = np.eye(d).reshape((d, d) + (1,) * d)
    GJ = I - GE
    GJ[(slice(None), slice(None)) + (0,) * d] = 0.0
    return GJ


def proj_U(shape):
    """G^U(k) = I at k = 0, 0 elsewhere (Def. projection)."""
    d = len(shape)
    G = np.zeros((d, d) + tuple(shape))
    G[(slice(None), slice(None)) + (0,) * d] = np.eye(d)
    return G


def apply_blockdiag(G, v):
    """(G v)(k) = G(k) v(k) for a block-diagonal field G (d, d, *s), v (d, *s)."""
    return np.einsum("ab...,b...->a...", G, v)


def inner(u, v):
    """L2 inner product of two fields given by Fourier coefficients (Parseval):
    Re sum_k u_hat(k) . conj(v_hat(k))."""
    return float(np.real(np.vdot(v, u)))
