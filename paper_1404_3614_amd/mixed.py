"""Mixed batches of uneven size: cells are grouped by size class (d, N, ncoef)
and every class is solved as one lockstep batch (one launch per pass covers
all cells of the class).

A class keeps its problem handles, workspaces and batch between calls, so a
stream of new cells of the same classes re-uses them through
hom_batch_update_coefficients.  Classes run on streams of their own, so
small classes overlap the large ones on the GPU, in one of three modes:
"graph": every class's primal and dual solves advance together from one
captured HIP graph per chunk of iterations (hom_group_solve_pair), one host
poll per chunk; "streams": every solve replays its own chunk graph on its own
stream, one host loop polls them all (no class waits for another's chunks);
"threads": each class's pair solve is driven by a host thread of its own.
"""
from __future__ import annotations

import time
from collections import OrderedDict
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import api


class MixedSolver:
    def __init__(self, precision="mixed", concurrent=True, stop="residual", etol=None, a_min=0.0, a_max=0.0,
                 mode="streams"):
        assert mode in ("graph", "streams", "threads")
        self.precision = precision
        self.concurrent = concurrent
        self.mode = mode
        self.stop = (stop, etol, a_min, a_max)   # Batch.set_stop arguments of every class
        self.classes = {}
        self._group = None                       # (class keys, api.Group) of the last graph-mode solve

    def _class(self, key, count, coefs):
        d, N, nc, Y = key
        cls = self.classes.get(key)
        if cls is None or len(cls["probs"]) != count:
            stream = torch.cuda.Stream()
            probs = [api.Problem(d, N, Y, Ah, Bh, precision=self.precision, ncoef=nc, stream=stream)
                     for (Ah, Bh) in coefs]
            cls = dict(probs=probs, batch=api.Batch(probs), stream=stream)
            cls["batch"].set_stop(*self.stop)
            # tile shapes are chosen now, on this thread, before classes run side by side
            for dual in (False, True):
                cls["batch"].tuning(dual, d)
            self.classes[key] = cls
        else:
            cls["batch"].update_coefficients(coefs)
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

    def solve(self, groups, n_total, tol=1e-6, maxit=20000, timings=None):
        """Bounds of every cell (list in input order) with per-cell iteration counts.
        timings: optional dict filled with the wall time of every class."""
        out = [None] * n_total
        # problem handles and batches are created here, on the calling thread
        work = [(key, items, self._class(key, len(items), [(Ah, Bh) for _, Ah, Bh in items]))
                for key, items in groups.items()]
        torch.cuda.synchronize()
        if self.mode in ("graph", "streams") and self.concurrent:
            keys = tuple(k for k, _, _ in work)
            batches = [cls["batch"] for _, _, cls in work]
            if self._group is None or self._group[0] != keys or \
                    any(a is not b for a, b in zip(self._group[1].batches, batches)):
                self._group = (keys, api.Group(batches))
                self._group[1].set_launch(self.mode)
            t0 = time.perf_counter()
            res_all = self._group[1].solve_bounds(tol=tol, maxit=maxit)
            dt = time.perf_counter() - t0
            for (key, items, cls), res in zip(work, res_all):
                if timings is not None:
                    timings[key] = dt
                for (i, _, _), r in zip(items, res):
                    r["class"] = dict(d=key[0], N=key[1])
                    out[i] = r
            return out

        def run(job):
            key, items, cls = job
            t0 = time.perf_counter()
            with torch.cuda.stream(cls["stream"]):
                res = cls["batch"].solve_bounds(tol=tol, maxit=maxit)
            cls["stream"].synchronize()
            return key, items, res, time.perf_counter() - t0

        if self.concurrent and len(work) > 1:
            with ThreadPoolExecutor(max_workers=min(len(work), 8)) as ex:
                done = list(ex.map(run, work))
        else:
            done = [run(w) for w in work]
        for key, items, res, dt in done:
            if timings is not None:
                timings[key] = dt
            for (i, _, _), r in zip(items, res):
                r["class"] = dict(d=key[0], N=key[1])
                out[i] = r
        return out

    def solve_timed(self, groups, n_total, tol=1e-6, maxit=20000):
        """As solve, but class after class on this thread with every kernel launched
        directly between HIP events (Batch.set_timing), so that the durations are
        those of each kernel alone.  Returns (results, {key: (ms per launch, launches)})."""
        out = [None] * n_total
        timing = {}
        for key, items in groups.items():
            cls = self._class(key, len(items), [(Ah, Bh) for _, Ah, Bh in items])
            b = cls["batch"]
            torch.cuda.synchronize()
            b.set_timing(True)
            with torch.cuda.stream(cls["stream"]):
                res = b.solve_bounds(tol=tol, maxit=maxit)
            cls["stream"].synchronize()
            timing[key] = b.get_timing()
            b.set_timing(False)
            for (i, _, _), r in zip(items, res):
                r["class"] = dict(d=key[0], N=key[1])
                out[i] = r
        return out, timing

