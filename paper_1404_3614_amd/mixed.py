"""Mixed batches of uneven size: cells are grouped by size class (d, N, ncoef)
and every class is solved as one lockstep batch (one launch per pass covers
all cells of the class, iterations replayed from a captured graph).

A class keeps its problem handles, workspaces and batch between calls, so a
stream of new cells of the same classes re-uses them through
hom_update_coefficients.
"""
from __future__ import annotations

from collections import OrderedDict

import numpy as np
import torch

from . import api


class MixedSolver:
    def __init__(self, precision="mixed", stream=None):
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.classes = {}

    def _class(self, key, count, coefs):
        d, N, nc, Y = key
        cls = self.classes.get(key)
        if cls is None or len(cls["probs"]) != count:
            probs = [api.Problem(d, N, Y, Ah, Bh, precision=self.precision, ncoef=nc, stream=self.stream)
                     for (Ah, Bh) in coefs]
            cls = dict(probs=probs, batch=api.Batch(probs))
            self.classes[key] = cls
        else:
            for p, (Ah, Bh) in zip(cls["probs"], coefs):
                p.update_coefficients(Ah, Bh)
        return cls

    def prepare(self, specs):
        """Fourier data of every cell (device), grouped by class.  specs: [(N, cell)]."""
        groups = OrderedDict()
        for i, (N, cell) in enumerate(specs):
            N = tuple(int(n) for n in (N if np.iterable(N) else [N] * cell.d))
            nc = api.cell_ncoef(cell)
            key = (cell.d, N, nc, tuple(float(y) for y in cell.Y))
            Ah, Bh, _ = api.coef_from_cell(cell, N, ncoef=nc)
            groups.setdefault(key, []).append((i, Ah, Bh))
        return groups

    def solve(self, groups, n_total, tol=1e-6, maxit=20000):
        """Bounds of every cell (list in input order) with per-cell iteration counts."""
        out = [None] * n_total
        for key, items in groups.items():
            cls = self._class(key, len(items), [(Ah, Bh) for _, Ah, Bh in items])
            res = cls["batch"].solve_bounds(tol=tol, maxit=maxit)
            for (i, _, _), r in zip(items, res):
                r["class"] = dict(d=key[0], N=key[1])
                out[i] = r
        return out
