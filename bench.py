"""Benchmark: guaranteed bound pairs per second on one MI355X.

Workload (default): 2D cells on an N = 313 grid (doubled grid 625 x 625), each a
random two-phase 125 x 125 pixel image (phase Bernoulli(0.5) per 5 x 5 block
of the doubled grid), a in {1, 100}; both unit loads; primal + dual CG to
relative residual 1e-6 in mixed precision (FP32 FFT/apply, FP64 CG and bound
quadrature).  One step = for every cell of the batch: the doubled-grid
coefficient setup (FP64 inverse FFT of the Fourier data of A and A^-1), the
right-hand sides, 2 primal + 2 dual solves and the FP64 bound evaluation.
Fourier data of the pixel images are computed on the device once, before the
timed region (inputs resident in HBM).

Prints one JSON line (see the design doc for the roofline and traffic method).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bound pairs/s at 1e-6 rel. tol (plain vs learned+batched CG); matvec HBM GB/s"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=32, help="cells per step")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cells", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true", help="skip the one-cell-at-a-time comparison leg")
    return ap.parse_args()


def c2_cell(i):
    import homgen
    return homgen.pixel_cell(1404002 + 7919 * i, P=125, values=(1.0, 100.0))


def apply_bytes(pb, nload):
    """Algorithmic bytes of one launch of the column pass: the pruned
    intermediate (N0 x M1 x M2 complex per pack) read once and written once, and
    the coefficient on the doubled grid read once."""
    d = pb.d
    N0 = pb.N[0]
    M = [2 * n - 1 for n in pb.N]
    plane = 1
    for m in M[1:]:
        plane *= m
    P = (nload * d + 1) // 2
    cs = 8 if pb.precision == "mixed" else 16
    rs = 4 if pb.precision == "mixed" else 8
    Mt = plane * M[0]
    return 2 * N0 * plane * P * cs + pb.ncoef * Mt * rs


def pass_bytes(pb, nload):
    """Algorithmic bytes per unit (one cell, nload loads) of each pass of one
    CG iteration (primal, m = 1 component per load):
      first: CG vectors x, p, r, s read and x, r written (FP64 complex on the
             stored half of Z_N) + the row-transformed intermediate written;
      apply: intermediate read and written + coefficient on the doubled grid read;
      last : intermediate read + r, p, s read and p, s written."""
    d = pb.d
    N = list(pb.N)
    M = [2 * n - 1 for n in N]
    H0 = (N[0] + 1) // 2
    S = H0
    for n in N[1:]:
        S *= n
    P = (nload * d + 1) // 2
    cs = 8 if pb.precision == "mixed" else 16
    vec = nload * 1 * S * 16
    inner = 1
    for n in N[1:-1]:
        inner *= n
    rowbuf = N[0] * inner * M[-1] * P * cs
    return dict(first=6 * vec + rowbuf, apply=apply_bytes(pb, nload), last=rowbuf + 5 * vec)


def cpu_baseline(ncells, tol):
    """The FP64 oracle on a bounded sample: ncells C2 bound pairs on the host."""
    import numpy as np
    from oracle import galerkin as ga, spectral as sp
    sp.WORKERS = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    for i in range(ncells):
        prob = ga.make_problem(c2_cell(i), 313)
        ga.bounds(prob, tol=tol)
    dt = time.perf_counter() - t0
    return dict(value=ncells / dt, unit="bound pairs/s", cores=sp.WORKERS, kind="oracle",
                sample=f"{ncells} C2 cell(s): setup + 2 primal + 2 dual FP64 CG solves to {tol:g} + bounds, "
                       f"{dt:.1f} s; scipy.fft with {sp.WORKERS} worker threads, other NumPy work single-threaded")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import api

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N = (313, 313)
    B = args.cells
    # inputs resident in HBM: Fourier data of A and A^-1 for every cell
    coefs = [H.coef_from_cell(c2_cell(i), N) for i in range(B)]
    stream = torch.cuda.Stream()
    # problem handles, workspaces and the batch (with its captured graphs) are built once;
    # every step loads the coefficients of its cells into them (a1) and solves
    probs = [H.Problem(2, N, (1.0, 1.0), Ah, Bh, precision=args.precision, ncoef=nc, max_loads=2, stream=stream)
             for (Ah, Bh, nc) in coefs]
    batch = H.Batch(probs)
    state = {"batch": batch, "probs": probs}

    pairs = [(Ah, Bh) for (Ah, Bh, nc) in coefs]

    def step():
        # a1: doubled-grid coefficients of every cell; a2-a10: lockstep CG of the batch; a8: bounds
        batch.update_coefficients(pairs)
        return batch.solve_bounds(tol=args.tol)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region 1 (value): CG iterations replayed from captured HIP graphs
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # timed region 2 (kernel durations for the roofline): the same steps, iterations launched
    # directly with HIP events around every kernel on the library stream
    batch.set_timing(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_events = time.perf_counter() - t1
    avg_ms, launches = batch.get_timing()
    batch.set_timing(False)
    res = results[-1]
    ms_per_step = 1e3 * dt / args.steps
    value = B * args.steps / dt
    iters = [i["iters"] for i in res[0]["info_primal"] + res[0]["info_dual"]]
    # unit-launches of the timed region: a cell stays in the lockstep launches
    # until all of its loads have stopped (iteration index + 1 launches)
    unit_launches = sum(max(i["iters"] for i in cell[key]) + 1
                        for r in results for cell in r for key in ("info_primal", "info_dual"))

    # plain CG for comparison: the same cells one at a time (one problem handle, no batching)
    nplain = 0 if args.no_plain else min(B, 4)
    if nplain:
        single = H.Problem(2, N, (1.0, 1.0), *coefs[0][:2], precision=args.precision, ncoef=coefs[0][2],
                           max_loads=2, stream=stream)
        single.solve_bounds(tol=args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nplain):
        single.update_coefficients(*coefs[i][:2])
        single.solve_bounds(tol=args.tol)
    torch.cuda.synchronize()
    plain_value = nplain / (time.perf_counter() - t0) if nplain else None

    # roofline of the dominant kernel, from the live event timings of the timed region
    pbytes = pass_bytes(probs[0], 2)
    total_ms = {k: avg_ms[k] * launches[k] for k in avg_ms}
    dom = max(total_ms, key=total_ms.get)
    nbytes = unit_launches * pbytes[dom] / max(launches[dom], 1)
    ms = avg_ms[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9
    names = dict(first="k_first (row pass: CG update, fields, inverse FFT of the last axis)",
                 apply="k_apply (column pass: inverse FFT, coefficient, forward FFT)",
                 last="k_last (row pass: forward FFT, projection, CG direction update)")
    per_pass = {}
    for k in ("first", "apply", "last"):
        if launches[k]:
            b = unit_launches * pbytes[k] / launches[k]
            per_pass[k] = dict(ms_per_launch=round(avg_ms[k], 5), bytes_per_launch=int(b),
                               gbs=round(b / (avg_ms[k] * 1e-3) / 1e9, 1), launches=launches[k])
    roofline = dict(bound="hbm", kernel=names[dom], achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None, bytes_per_launch=int(nbytes),
                    ms_per_launch=round(ms, 5), per_pass=per_pass,
                    bytes_model="pass_bytes() in bench.py; units per launch = active cells of the batch",
                    timed_region="second timed pass of the same steps, kernels launched directly by "
                                 "hipExtLaunchKernelGGL with start/stop HIP events on the library stream",
                    value_events_pass=round(B * args.steps / dt_events, 3))

    line = dict(metric=METRIC, value=round(value, 3), unit="bound pairs/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32 FFT/apply + f64 CG/bounds" if args.precision == "mixed" else "f64",
                data="synthetic",
                config=dict(workload="C2: 2D N=313 (doubled grid 625^2), random two-phase 125x125 pixel image, "
                                     "a in {1,100}, both loads, primal+dual, batched lockstep CG",
                            cells_per_step=B, tol=args.tol, precision=args.precision, cg_iters=iters,
                            batched="all cells of a step in lockstep (one launch per pass covers every cell)",
                            plain_bound_pairs_per_s=None if plain_value is None else round(plain_value, 3),
                            tile_tuning=dict(primal=batch.tuning(False, 2), dual=batch.tuning(True, 2))),
                roofline=roofline)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_cells, args.tol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
