"""Seeded synthetic microstructures (geometry only).

This module is shared by the FP64 oracle and by the GPU library's Python
binding.  It draws random geometry and phase values and returns plain
descriptors; it performs none of the homogenization arithmetic (no Fourier
coefficients, no grids, no solves).  Every generator takes an integer seed and
uses ``numpy.random.default_rng`` (PCG64), so both sides see bit-identical
inputs.

Descriptors
-----------
``Inclusions``  -- a matrix phase with coefficient ``A0`` (d x d, SPD) plus
    non-overlapping inclusions, each of kind ``"rect"`` (axis-aligned box with
    side lengths ``size``) or ``"ball"`` (radius ``size[0]``), centred at
    ``center``, with constant coefficient ``A`` inside (d x d, SPD).  This is the
    matrix-inclusion medium of Section 6 (eq. A_with_inclusions) with indicator
    topologies, where inside inclusion j the coefficient is the inclusion's own
    value.
``Pixels``      -- a pixel/voxel image on P_1 x ... x P_d cells of the unit cell;
    ``phase`` holds an integer phase id per pixel and ``phase_A`` the d x d
    coefficient of each phase.  Pixel i along axis a covers
    [-Y_a/2 + i*Y_a/P_a, -Y_a/2 + (i+1)*Y_a/P_a).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np

__all__ = [
    "Inclusions", "Pixels", "square_inclusion_cell", "laminate_cell",
    "pixel_cell", "sphere_cell", "random_squares_cell", "random_spheres_cell",
    "random_spd", "batch_specs", "homogeneous_cell", "foam_cell",
]


@dataclass
class Inclusions:
    d: int
    Y: np.ndarray                      # (d,) cell side lengths
    A0: np.ndarray                     # (d, d) matrix phase
    kind: list = field(default_factory=list)      # "rect" | "ball" per inclusion
    center: list = field(default_factory=list)    # (d,) arrays
    size: list = field(default_factory=list)      # (d,) side lengths, or (1,) radius
    A: list = field(default_factory=list)         # (d, d) arrays

    def add(self, kind, center, size, A):
        self.kind.append(kind)
        self.center.append(np.asarray(center, dtype=np.float64))
        self.size.append(np.atleast_1d(np.asarray(size, dtype=np.float64)))
        self.A.append(np.asarray(A, dtype=np.float64))
        return self

    @property
    def n(self):
        return len(self.kind)


@dataclass
class Pixels:
    d: int
    Y: np.ndarray          # (d,)
    phase: np.ndarray      # int array, shape (P_1, ..., P_d)
    phase_A: np.ndarray    # (nphase, d, d)


def _eye(d, s=1.0):
    return s * np.eye(d)


def homogeneous_cell(d, A0, Y=None):
    Y = np.ones(d) if Y is None else np.asarray(Y, float)
    return Inclusions(d=d, Y=Y, A0=np.asarray(A0, float))


def square_inclusion_cell(d=2, side=0.5, rho_in=10.0, Y=None):
    """Centred square/cube inclusion of coefficient rho_in*I in an I matrix."""
    Y = np.ones(d) if Y is None else np.asarray(Y, float)
    c = Inclusions(d=d, Y=Y, A0=_eye(d))
    c.add("rect", np.zeros(d), np.full(d, side) * Y, _eye(d, rho_in))
    return c


def laminate_cell(d=2, h=0.5, rho=10.0, Y=None):
    """Layer of thickness h along axis 1 (full extent in the others)."""
    Y = np.ones(d) if Y is None else np.asarray(Y, float)
    c = Inclusions(d=d, Y=Y, A0=_eye(d))
    size = Y.copy()
    size[0] = h
    c.add("rect", np.zeros(d), size, _eye(d, rho))
    return c


def pixel_cell(seed, P=125, values=(1.0, 100.0), d=2, p_inclusion=0.5):
    """Random two-phase pixel image: phase 1 with probability p_inclusion."""
    rng = np.random.default_rng(seed)
    phase = (rng.random((P,) * d) < p_inclusion).astype(np.int32)
    phase_A = np.stack([_eye(d, values[0]), _eye(d, values[1])])
    return Pixels(d=d, Y=np.ones(d), phase=phase, phase_A=phase_A)


def _periodic_dist(a, b, Y):
    dlt = a - b
    dlt -= Y * np.round(dlt / Y)
    return dlt


def random_spd(rng, d, lo=0.1, hi=10.0):
    """Q diag(lambda) Q^T with log-uniform eigenvalues and a Haar rotation."""
    lam = np.exp(rng.uniform(math.log(lo), math.log(hi), size=d))
    Z = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(Z)
    Q = Q * np.sign(np.diag(R))
    S = (Q * lam) @ Q.T
    return 0.5 * (S + S.T)


def _place_spheres(rng, n, rmin, rmax, Y, max_tries=100000):
    centers, radii = [], []
    tries = 0
    while len(centers) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place non-overlapping spheres")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(-0.5, 0.5, size=3) * Y
        ok = all(np.linalg.norm(_periodic_dist(c, c2, Y)) > r + r2
                 for c2, r2 in zip(centers, radii))
        if ok:
            centers.append(c)
            radii.append(r)
    return centers, radii


def sphere_cell(seed, n=20, rmin=0.08, rmax=0.15, rho=10.0, anisotropic=False):
    """Non-overlapping (periodic minimum image) spheres in an I matrix.

    anisotropic=False: every sphere has rho*I.  anisotropic=True: every sphere
    gets its own SPD matrix Q diag(lambda) Q^T, lambda log-uniform in [0.1, 10].
    The geometry is the same for both variants of a given seed.
    """
    rng = np.random.default_rng(seed)
    Y = np.ones(3)
    centers, radii = _place_spheres(rng, n, rmin, rmax, Y)
    rng_m = np.random.default_rng(seed + 7919)
    c = Inclusions(d=3, Y=Y, A0=_eye(3))
    for ctr, r in zip(centers, radii):
        A = random_spd(rng_m, 3) if anisotropic else _eye(3, rho)
        c.add("ball", ctr, [r], A)
    return c


def random_squares_cell(seed, kmin=1, kmax=10, smin=0.05, smax=0.3,
                        logrho=(math.log10(2.0), 3.0), max_tries=100000):
    """2D: K ~ U{kmin..kmax} non-overlapping axis-aligned squares, rho*I."""
    rng = np.random.default_rng(seed)
    Y = np.ones(2)
    K = int(rng.integers(kmin, kmax + 1))
    rho = 10.0 ** rng.uniform(*logrho)
    c = Inclusions(d=2, Y=Y, A0=_eye(2))
    cs, hs = [], []
    tries = 0
    while len(cs) < K:
        tries += 1
        if tries > max_tries:
            break
        h = rng.uniform(smin, smax)
        ctr = rng.uniform(-0.5, 0.5, size=2)
        ok = True
        for c2, h2 in zip(cs, hs):
            dl = np.abs(_periodic_dist(ctr, c2, Y))
            if np.all(dl < 0.5 * (h + h2) + 1e-9):
                ok = False
                break
        if ok:
            cs.append(ctr)
            hs.append(h)
    for ctr, h in zip(cs, hs):
        c.add("rect", ctr, [h, h], _eye(2, rho))
    return c, rho


def random_spheres_cell(seed, kmin=5, kmax=20, rmin=0.08, rmax=0.15,
                        logrho=(math.log10(2.0), 3.0)):
    """3D: K ~ U{kmin..kmax} non-overlapping spheres of rho*I."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(kmin, kmax + 1))
    rho = 10.0 ** rng.uniform(*logrho)
    centers, radii = _place_spheres(rng, K, rmin, rmax, np.ones(3))
    c = Inclusions(d=3, Y=np.ones(3), A0=_eye(3))
    for ctr, r in zip(centers, radii):
        c.add("ball", ctr, [r], _eye(3, rho))
    return c, rho


def batch_specs(seed0=1404004, n2d=512, n3d=64, Ns2d=(13, 41, 63, 313), N3d=41,
                logrho=(math.log10(2.0), 3.0)):
    """Mixed batch: n2d random-square 2D cells with N drawn from Ns2d and n3d
    random-sphere 3D cells at N3d.  Returns a list of (N, cell, rho)."""
    out = []
    for i in range(n2d):
        rng = np.random.default_rng(seed0 + i)
        N = int(rng.choice(np.asarray(Ns2d)))
        cell, rho = random_squares_cell(seed0 + 100000 + i, logrho=logrho)
        out.append((N, cell, rho))
    for i in range(n3d):
        cell, rho = random_spheres_cell(seed0 + 200000 + i, logrho=logrho)
        out.append((N3d, cell, rho))
    return out


def foam_cell(seed, P=1200, porosity=0.5, rmin=0.01, rmax=0.04, values=(0.029, 0.49)):
    """Foam-like two-phase pixel image on P x P pixels of the unit cell: a
    solid phase (phase 1, coefficient values[1]) with overlapping circular
    pores (phase 0, values[0]) of radii uniform in [rmin, rmax], centres
    uniform, periodic, added until the pore fraction reaches `porosity`.  The
    default coefficients are the thermal conductivities of fly ash and air of
    the paper's foam example."""
    rng = np.random.default_rng(seed)
    c = (np.arange(P) + 0.5) / P - 0.5               # pixel centres on (-1/2, 1/2)
    solid = np.ones((P, P), dtype=bool)
    target = int(round(porosity * P * P))
    pores = 0
    while pores < target:
        cx, cy = rng.random(2) - 0.5
        r = rng.uniform(rmin, rmax)
        h = int(math.ceil(r * P)) + 1
        i0 = int(math.floor((cx + 0.5) * P))
        j0 = int(math.floor((cy + 0.5) * P))
        ii = np.arange(i0 - h, i0 + h + 1) % P
        jj = np.arange(j0 - h, j0 + h + 1) % P
        dx = c[ii] - cx
        dx -= np.round(dx)
        dy = c[jj] - cy
        dy -= np.round(dy)
        inside = dx[:, None] ** 2 + dy[None, :] ** 2 < r * r
        sub = solid[np.ix_(ii, jj)]
        pores += int(np.count_nonzero(sub & inside))
        sub &= ~inside
        solid[np.ix_(ii, jj)] = sub
    phase_A = np.stack([_eye(2, values[0]), _eye(2, values[1])])
    return Pixels(d=2, Y=np.ones(2), phase=solid.astype(np.int32), phase_A=phase_A)
