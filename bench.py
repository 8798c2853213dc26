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
    ap.add_argument("--cells", type=int, default=8, help="cells per step")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cells", type=int, default=1)
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
    probs = [None] * B

    def step():
        out = []
        for i in range(B):
            Ah, Bh, nc = coefs[i]
            pb = H.Problem(2, N, (1.0, 1.0), Ah, Bh, precision=args.precision, ncoef=nc, max_loads=2,
                           stream=stream)
            b = pb.solve_bounds(tol=args.tol)
            probs[i] = pb
            out.append(b)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    value = B * args.steps / dt
    iters = [i["iters"] for i in res[0]["info_primal"] + res[0]["info_dual"]]

    # per-kernel durations on the library stream, same launch configuration as the solves
    pb = probs[0]
    prof = pb.profile_passes(dual=False, nload=2, reps=50)
    dom = max(prof, key=prof.get)
    ms = prof["apply"]
    nbytes = apply_bytes(pb, 2)
    achieved = nbytes / (ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel="k_apply (column pass: inverse FFT, coefficient, forward FFT)",
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_launch=nbytes, ms_per_launch=round(ms, 5), dominant=dom,
                    passes_ms={k: round(v, 5) for k, v in prof.items()})

    line = dict(metric=METRIC, value=round(value, 3), unit="bound pairs/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32 FFT/apply + f64 CG/bounds" if args.precision == "mixed" else "f64",
                data="synthetic",
                config=dict(workload="C2: 2D N=313 (doubled grid 625^2), random two-phase 125x125 pixel image, "
                                     "a in {1,100}, both loads, primal+dual, plain CG one cell at a time",
                            cells_per_step=B, tol=args.tol, precision=args.precision, cg_iters=iters),
                roofline=roofline)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_cells, args.tol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
