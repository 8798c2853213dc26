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

Other workloads (--workload): c4, a mixed batch of 512 2D cells of uneven N
(13, 41, 63, 313) and 64 3D cells (N = 41), random inclusions with contrast
log-uniform in [2, 1e3], solved class by class in lockstep batches; c5, the
learned initial guess (U-Net trained on solver fields of 2D N = 63 cells),
plain versus learned + batched on held-out cells of contrast 1e2 - 1e3; e1
and e2, the paper's square experiments on odd grids N = 5 3^j and on even
GaNi grids n = 2^j (Ga and the paper's Algorithm per grid, FP64); e3, a
synthetic stand-in of the paper's 1200^2 foam image.

Prints one JSON line.  The roofline object divides the algorithmic bytes per
launch of the dominant kernel by its duration measured with HIP events; its
traffic field is the HBM traffic per launch from the hardware counters of a
committed profile, reported only while the kernel sources are the ones that
profile measured.
"""
from __future__ import annotations

import argparse
import gc
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
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=32, help="cells per step")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-cells", type=int, default=2, help="C2 cells the CPU oracle solves (about 6 s each)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-cell-at-a-time comparison leg")
    ap.add_argument("--no-energy", action="store_true", help="skip the guaranteed-energy-rule leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 leg of the same cells")
    ap.add_argument("--theta", type=float, default=1e-2,
                    help="gap rule: each bound's algebraic error below theta times the discretisation gap")
    ap.add_argument("--tiles", default=None,
                    help="pin the FP32 tile shape: row_pairs,row_threads,apply_points,apply_half_exchange,"
                         "apply_all_packs")
    ap.add_argument("--stop", default="residual", choices=["residual", "energy", "guaranteed", "gap"],
                    help="stopping rule: the residual rule at --tol, or that rule or an energy rule at --etol "
                         "(energy: extrapolated tail; guaranteed: Gauss-Radau bound)")
    ap.add_argument("--etol", type=float, default=1e-7,
                    help="energy rules: remaining energy decrease / energy of the iterate")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "e1", "e2", "e3"])
    ap.add_argument("--c3-cells", type=int, default=64, help="c3: cells per batch (C3a and C3b each)")
    ap.add_argument("--c3-variant", default="both", choices=["both", "a", "b"],
                    help="c3: isotropic C3a, anisotropic C3b or both (the value is C3a's whenever it runs)")
    ap.add_argument("--c4-mode", default="streams", choices=["graph", "streams", "threads"],
                    help="c4: one captured graph for all classes per chunk, every solve's own graph from one "
                         "host loop, or a host thread per class")
    ap.add_argument("--e1-jmax", type=int, default=5, help="e1: grids N = 5 3^j for j <= jmax")
    ap.add_argument("--e2-jmax", type=int, default=9, help="e2: even grids n = 2^j for 2 <= j <= jmax")
    ap.add_argument("--c5-train", type=int, default=16384, help="c5: 2D training cells (0: no 2D class)")
    ap.add_argument("--c5-steps", type=int, default=3000, help="c5: Adam steps of the 2D network (batch 16)")
    ap.add_argument("--c5-test", type=int, default=256, help="c5: held-out 2D cells")
    ap.add_argument("--c5-train3d", type=int, default=4096, help="c5: 3D training cells (0: no 3D class)")
    ap.add_argument("--c5-steps3d", type=int, default=1500, help="c5: Adam steps of the 3D network (batch 2)")
    ap.add_argument("--c5-test3d", type=int, default=64, help="c5: held-out 3D cells")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_hbm_traffic.md")
KERNEL_SOURCES = ["paper_1404_3614_amd/csrc/hom_fast.hip", "paper_1404_3614_amd/csrc/hom_regfft.hpp",
                  "paper_1404_3614_amd/csrc/hom_device.hpp", "paper_1404_3614_amd/csrc/hom_internal.hpp"]


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tiles):
    """HBM bytes per launch of the three CG passes from the committed counter
    profile, or None when the kernel sources or the tile shape differ from
    the ones it measured."""
    try:
        txt = open(TRAFFIC_FILE).read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != kernel_source_digest() or blob.get("tiles") != tiles:
        return None
    return blob.get("bytes_per_launch")


GOLDEN = os.path.join(ROOT, "tests", "golden", "reference_bounds.json")


def golden(name):
    """Oracle bounds (CG to 1e-11) of a configuration, written by oracle/make_golden.py."""
    import numpy as np
    try:
        with open(GOLDEN) as f:
            g = json.load(f)[name]
    except (OSError, KeyError, ValueError):
        return None
    return {k: np.array(g[k]) for k in ("A_up", "A_low")}


def bound_error(res, ref):
    """Relative bound error max_ab |X - X_ref|_ab / ||X_ref||_2 for X in {upper, lower}."""
    import numpy as np
    if ref is None:
        return None
    return {k: float(np.abs(res[k] - ref[k]).max() / np.linalg.norm(ref[k], 2)) for k in ("A_up", "A_low")}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


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


def pass_bytes(pb, nload, plane=False, m=1):
    """Algorithmic bytes per unit (one cell, nload loads) of each pass of one
    CG iteration (m components of the unknown per load: 1 primal and 2D dual,
    2 for the 3D dual):
      first  : CG vectors x, p, r, s read and x, r written (FP64 complex on the
               stored half of Z_N) + the row-transformed intermediate written
               (N0 x N1 x M2 per pack; 2D: N0 x M1);
      mid_inv: (3D) that intermediate read, N0 x M1 x M2 written;
      apply  : intermediate (N0 x M1 x M2) read and written + coefficient on the
               doubled grid read;
      mid_fwd: (3D) N0 x M1 x M2 read, N0 x N1 x M2 written;
      last   : row intermediate read + r, p, s read and p, s written.
    plane (3D plane pass in place of mid_inv, apply and mid_fwd): the row
    intermediate read and written + the coefficient on the doubled grid read."""
    d = pb.d
    N = list(pb.N)
    M = [2 * n - 1 for n in N]
    H0 = (N[0] + 1) // 2
    S = H0
    for n in N[1:]:
        S *= n
    P = (nload * d + 1) // 2
    cs = 8 if pb.precision == "mixed" else 16
    vec = nload * m * S * 16
    inner = 1
    for n in N[1:-1]:
        inner *= n
    rowbuf = N[0] * inner * M[-1] * P * cs
    out = dict(first=6 * vec + rowbuf, apply=apply_bytes(pb, nload), last=rowbuf + 5 * vec)
    if d == 3 and plane:
        Mt = M[0] * M[1] * M[2]
        out["apply"] = 2 * rowbuf + pb.ncoef * Mt * (4 if pb.precision == "mixed" else 8)
    elif d == 3:
        full = N[0] * M[1] * M[2] * P * cs
        out.update(mid_inv=rowbuf + full, mid_fwd=full + rowbuf)
    return out


def survey_matvec_bytes(pb, nload):
    """The minimum bytes of one operator application to the nload loads of a
    cell: the coefficient on the doubled grid read once (FP32 in mixed mode,
    FP64 otherwise) and, per load, the FP64 potential coefficients of Z_N read
    and the result written (N^d reals each: the stored half of the complex
    spectrum)."""
    Mt, Nt = 1, 1
    for n in pb.N:
        Mt *= 2 * n - 1
        Nt *= n
    rs = 4 if pb.precision == "mixed" else 8
    return pb.ncoef * Mt * rs + nload * 2 * Nt * 8


# FP32 flops of the column pass as executed (a multiply-add counts 2).  The
# register DFTs are built as small expression graphs with the same zero
# propagation and dead-output removal as the kernels: inputs of the first
# inverse DFT that lie outside Z_N are zero, outputs of the last forward DFT
# outside Z_N are dropped.  Costs: complex add/sub 2, scale 2, multiply-add 4,
# compile-time rotation 6, run-time twiddle 6, multiply by i 0.
SPLIT = {9: (3, 3), 25: (5, 5), 81: (9, 9), 125: (25, 5), 625: (25, 25)}


class _Dag:
    def __init__(self):
        self.cost, self.args = [], []

    def node(self, cost, *args):
        self.cost.append(cost)
        self.args.append(args)
        return len(self.cost) - 1

    def add(self, a, b, sub=False):
        if a is None and b is None:
            return None
        if a is None:
            return b if not sub else self.node(0, b)      # a negation folds into later operations
        if b is None:
            return a
        return self.node(2, a, b)

    def scl(self, a):
        return None if a is None else self.node(2, a)

    def axpy(self, acc, t):
        if t is None:
            return acc
        if acc is None:
            return self.node(2, t)
        return self.node(4, acc, t)

    def count(self, outs):
        seen, stack, total = set(), [o for o in outs if o is not None], 0
        while stack:
            n = stack.pop()
            if n in seen:
                continue
            seen.add(n)
            total += self.cost[n]
            stack.extend(self.args[n])
        return total


def _dft(g, x):
    n = len(x)
    if n == 1:
        return list(x)
    if n == 3:
        t = g.add(x[1], x[2])
        m = g.axpy(x[0], t)
        j = g.scl(g.add(x[1], x[2], sub=True))
        return [g.add(x[0], t), g.add(m, j), g.add(m, j, sub=True)]
    if n == 5:
        t1, t2 = g.add(x[1], x[4]), g.add(x[2], x[3])
        t3, t4 = g.add(x[1], x[4], sub=True), g.add(x[2], x[3], sub=True)
        b1 = g.axpy(g.axpy(x[0], t1), t2)
        b2 = g.axpy(g.axpy(x[0], t1), t2)
        j1 = g.axpy(g.scl(t3), t4)
        j2 = g.axpy(g.scl(t3), t4)
        return [g.add(x[0], g.add(t1, t2)), g.add(b1, j1), g.add(b2, j2), g.add(b2, j2, sub=True),
                g.add(b1, j1, sub=True)]
    n1, n2 = SPLIT[n]
    t = {}
    for b in range(n2):
        a = _dft(g, [x[n2 * i + b] for i in range(n1)])
        for k1 in range(n1):
            t[b, k1] = a[k1] if (b * k1) % n == 0 or a[k1] is None else g.node(6, a[k1])
    out = [None] * n
    for k1 in range(n1):
        bb = _dft(g, [t[b, k1] for b in range(n2)])
        for k2 in range(n2):
            out[k1 + n1 * k2] = bb[k2]
    return out


def _dead_row(M, n1):
    a, b = SPLIT[M]
    h = (M + 1) // 2 // 2
    return b * n1 > h and b * n1 + b - 1 < M - h


def column_line_flops(M):
    """Flops of one line as executed (inverse transform, forward transform,
    run-time twiddles; no coefficient), and those of the unpruned transforms."""
    a, b = SPLIT[M]

    def cnt(ins, keep=None):
        g = _Dag()
        out = _dft(g, [g.node(0) if i else None for i in ins])
        return g.count([o for i, o in enumerate(out) if keep is None or keep[i]])

    live = [not _dead_row(M, i) for i in range(a)]
    inv_first, fwd_last = cnt(live), cnt([True] * a, live)
    full_a, full_b = cnt([True] * a), cnt([True] * b)
    twiddles = 6 * M
    pruned = b * inv_first + a * full_b + a * full_b + b * fwd_last + 2 * twiddles
    return pruned, 2 * (b * full_a + a * full_b) + 2 * twiddles


def apply_flops(pb, nload):
    """FP32 flops per unit of the 2D column pass as executed: per point of the
    row axis and pack, the pruned inverse and forward length-M0 transforms and
    the coefficient product (2 flops per complex value isotropic, 6 otherwise)."""
    M = [2 * n - 1 for n in pb.N]
    P = (nload * pb.d + 1) // 2
    coef = 2 if pb.ncoef == 1 else 6
    lines = 1
    for m in M[1:]:
        lines *= m
    return lines * P * (column_line_flops(M[0])[0] + coef * M[0])


def plane_flops(pb, nload):
    """FP32 flops per unit of the 3D plane pass as executed: per plane m2 and
    pack, N0 lines along axis 1 and M1 columns along axis 0, each a pruned
    inverse and forward length-M transform (the column pass's line), and the
    isotropic coefficient product (2 flops per complex value) on M0 x M1 points."""
    M = [2 * n - 1 for n in pb.N]
    P = (nload * pb.d + 1) // 2
    return M[2] * P * ((pb.N[0] + M[1]) * column_line_flops(M[0])[0] + 2 * M[0] * M[1])


# FP32 vector peak of the chip: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed FP32) x 2.4 GHz =
# 157.3 TFLOP/s; without packed FP32 instructions (this build emits none) half of it
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
VALU_UNPACKED_TFLOPS = VALU_PEAK_TFLOPS / 2


def cpu_baseline(ncells, tol, gpu_results=None):
    """The FP64 oracle on a bounded sample: ncells C2 bound pairs on the host
    (and the GPU bounds of the same cells against it)."""
    from oracle import galerkin as ga, spectral as sp
    sp.WORKERS = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    errs = []
    for i in range(ncells):
        prob = ga.make_problem(c2_cell(i), 313)
        ref = ga.bounds(prob, tol=tol)
        if gpu_results is not None and i < len(gpu_results):
            errs.append(bound_error(gpu_results[i], ref))
    dt = time.perf_counter() - t0
    out = dict(value=ncells / dt, unit="bound pairs/s", cores=sp.WORKERS, kind="oracle",
               sample=f"{ncells} C2 cell(s): setup + 2 primal + 2 dual FP64 CG solves to {tol:g} + bounds, "
                      f"{dt:.1f} s; scipy.fft with {sp.WORKERS} worker threads, other NumPy work single-threaded",
               cpu_model=cpu_model(), host_cpus=os.cpu_count())
    if errs:
        out["gpu_bound_diff_vs_this_oracle_run"] = dict(
            A_up=max(e["A_up"] for e in errs), A_low=max(e["A_low"] for e in errs),
            note="both sides stop at the same residual tolerance; the reference at 1e-11 is in "
                 "config.bound_error_vs_oracle")
    return out


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
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "e1":
        return run_e1(args)
    if args.workload == "e2":
        return run_e2(args)
    if args.workload == "e3":
        return run_e3(args)
    N = (313, 313)
    B = args.cells
    # measured streaming peak of the device (project copy kernel, 4 GiB: well beyond the 256 MB
    # cache), beside the published HBM peak
    probe_gbs = H.probe_copy_gbs(1 << 32, reps=5)
    # inputs resident in HBM: Fourier data of A and A^-1 for every cell
    coefs = [H.coef_from_cell(c2_cell(i), N) for i in range(B)]
    stream = torch.cuda.Stream()
    # problem handles, workspaces and the batch (with its captured graphs) are built once;
    # every step loads the coefficients of its cells into them (a1) and solves
    probs = [H.Problem(2, N, (1.0, 1.0), Ah, Bh, precision=args.precision, ncoef=nc, max_loads=2, stream=stream)
             for (Ah, Bh, nc) in coefs]
    batch = H.Batch(probs)
    if args.tiles:
        r, t, a, x, al = (int(v) for v in args.tiles.split(","))
        for dual in (False, True):
            batch.set_tiles(dual, 2, row_pairs=r, row_threads=t, apply_points=a, apply_half_exchange=x,
                            apply_all_packs=al)

    # eigenvalue range of the phases (a in {1, 100}): the spectrum bound of the guaranteed rule
    a_min, a_max = H.cell_eig_range(c2_cell(0))
    batch.set_stop(args.stop, args.etol, a_min, a_max)
    pairs = [(Ah, Bh) for (Ah, Bh, nc) in coefs]

    def step():
        # a1: doubled-grid coefficients of every cell; a2-a10: lockstep CG of the batch; a8: bounds
        batch.update_coefficients(pairs)
        return batch.solve_bounds(tol=args.tol)

    # warm-up: the first step tunes the tile shapes and captures the graphs; then long-lived
    # objects (modules, handles, inputs) leave the cyclic collector's generations, so a full
    # collection cannot stall a timed step, and the remaining warm-up steps follow, so that the
    # timed region starts on a busy GPU
    for w in range(args.warmup):
        step()
        if w == 0:
            torch.cuda.synchronize()
            gc.collect()
            gc.freeze()
    torch.cuda.synchronize()
    if args.warmup == 0:
        gc.collect()
        gc.freeze()
    # timed region 1 (value): CG iterations replayed from captured HIP graphs
    t0 = time.perf_counter()
    results, step_ms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        results.append(step())
        step_ms.append(round(1e3 * (time.perf_counter() - ts), 2))
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

    # the guaranteed energy rule on the same steps (when the residual rule set the value):
    # bounds within a relative etol of their converged values, in fewer iterations
    energy_leg = gap_leg = None
    if args.stop == "residual" and not args.no_energy:
        batch.set_stop("guaranteed", args.etol, a_min, a_max)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res_e = step()
        torch.cuda.synchronize()
        dt_e = time.perf_counter() - t0
        batch.set_stop("residual")
        diff = max(max(float(np.abs(a[k] - b[k]).max() / np.linalg.norm(b[k], 2)) for k in ("A_up", "A_low"))
                   for a, b in zip(res_e, results[-1]))
        # the gap rule: each bound within theta of the discretisation gap of its entry
        batch.set_stop("gap", args.theta, a_min, a_max)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res_g = step()
        torch.cuda.synchronize()
        dt_g = time.perf_counter() - t0
        batch.set_stop("residual")
        ref_c2 = golden("C2")
        gap_leg = dict(rule="gap", theta=args.theta, bound_pairs_per_s=round(B * args.steps / dt_g, 3),
                       cg_iters=[i["iters"] for i in res_g[0]["info_primal"] + res_g[0]["info_dual"]],
                       bound_error_vs_oracle=bound_error(res_g[0], ref_c2),
                       gap_vs_oracle=None if ref_c2 is None else
                       float(np.abs(np.diag(ref_c2["A_up"]) - np.diag(ref_c2["A_low"])).max()),
                       definition="residual rule at tol, or each side's Gauss-Radau bound on its remaining error "
                                  "below theta times a guaranteed lower bound on the converged gap of its "
                                  "diagonal entry (primal and dual read each other's state chunk by chunk)")
        energy_leg = dict(rule="guaranteed", etol=args.etol, a_min=a_min, a_max=a_max,
                          bound_pairs_per_s=round(B * args.steps / dt_e, 3),
                          cg_iters=[i["iters"] for i in res_e[0]["info_primal"] + res_e[0]["info_dual"]],
                          max_rel_bound_diff_vs_residual_rule=diff,
                          definition="residual rule at tol, or the Gauss-Radau bound on the remaining energy "
                                     "(spectrum bound from the phases' eigenvalue range) below etol times the "
                                     "energy of the iterate, whichever first")

    # bound error of cell 0 (the C2 cell of the golden file) against the oracle (CG to 1e-11)
    err_mixed = bound_error(results[-1][0], golden("C2"))

    # the same cells in all-FP64 (FP64 transforms and coefficient), batched the same way
    fp64_leg = None
    if not args.no_fp64 and args.precision == "mixed":
        probs64 = [H.Problem(2, N, (1.0, 1.0), Ah, Bh, precision="fp64", ncoef=nc, max_loads=2, stream=stream)
                   for (Ah, Bh, nc) in coefs]
        batch64 = H.Batch(probs64)

        def step64():
            batch64.update_coefficients(pairs)
            return batch64.solve_bounds(tol=args.tol)

        step64()
        torch.cuda.synchronize()
        n64 = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(n64):
            res64 = step64()
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        fp64_leg = dict(bound_pairs_per_s=round(B * n64 / dt64, 3), steps=n64,
                        ms_per_step=round(1e3 * dt64 / n64, 3),
                        cg_iters=[i["iters"] for i in res64[0]["info_primal"] + res64[0]["info_dual"]],
                        bound_error_vs_oracle=bound_error(res64[0], golden("C2")),
                        max_rel_bound_diff_vs_mixed=max(
                            max(float(np.abs(a[k] - b[k]).max() / np.linalg.norm(b[k], 2)) for k in ("A_up", "A_low"))
                            for a, b in zip(results[-1], res64)))
        del batch64, probs64

    # plain CG for comparison: the same cells one at a time (one problem handle, no batching)
    nplain = 0 if args.no_plain else min(B, 4)
    if nplain:
        single = H.Problem(2, N, (1.0, 1.0), *coefs[0][:2], precision=args.precision, ncoef=coefs[0][2],
                           max_loads=2, stream=stream)
        single.set_stop(args.stop, args.etol, a_min, a_max)
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
    names = dict(first="k_first_fast (row pass: CG update, fields, inverse FFT of the last axis)",
                 apply="k_apply2_fast (column pass: inverse FFT, coefficient, forward FFT)",
                 last="k_last_fast (row pass: forward FFT, projection, CG direction update)")
    per_pass = {}
    for k in ("first", "apply", "last"):
        if launches[k]:
            b = unit_launches * pbytes[k] / launches[k]
            per_pass[k] = dict(ms_per_launch=round(avg_ms[k], 5), bytes_per_launch=int(b),
                               gbs=round(b / (avg_ms[k] * 1e-3) / 1e9, 1), launches=launches[k])
    aflops = unit_launches * apply_flops(probs[0], 2) / max(launches["apply"], 1)
    per_pass["apply"]["flops_per_launch"] = int(aflops)
    per_pass["apply"]["tflops"] = round(aflops / (avg_ms["apply"] * 1e-3) / 1e12, 2)
    tuning = dict(primal=batch.tuning(False, 2), dual=batch.tuning(True, 2))
    keys = ("row_pairs", "row_threads", "apply_points", "apply_half_exchange", "apply_all_packs")
    shape = [tuning["primal"][k] for k in keys]
    same_shape = all(tuning["dual"][k] == tuning["primal"][k] for k in keys)
    traffic_all = measured_traffic(shape) if same_shape else None
    traffic = None if traffic_all is None else traffic_all.get(dom)
    nbytes = unit_launches * pbytes[dom] / max(launches[dom], 1)
    ms = avg_ms[dom]
    hbm = dict(achieved=round(nbytes / (ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), bytes_per_launch=int(nbytes),
               traffic=traffic)
    it_bytes = sum(per_pass[k]["bytes_per_launch"] for k in per_pass)
    it_ms = sum(per_pass[k]["ms_per_launch"] for k in per_pass)
    matvec = dict(bytes_per_iteration=int(it_bytes), ms_per_iteration=round(it_ms, 5),
                  gbs=round(it_bytes / (it_ms * 1e-3) / 1e9, 1),
                  frac=round(it_bytes / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  measured_peak_gbs=round(probe_gbs, 1),
                  frac_of_measured=round(it_bytes / (it_ms * 1e-3) / 1e9 / probe_gbs, 4),
                  measured_peak_probe="hom_probe_copy: 4 GiB device copy, bytes read plus written")
    common = dict(kernel=names[dom], ms_per_launch=round(ms, 5), traffic=traffic, traffic_unit="bytes/launch",
                  traffic_per_pass=traffic_all, per_pass=per_pass, matvec=matvec,
                  bytes_model="pass_bytes() in bench.py; units per launch = active cells of the batch",
                  timed_region="second timed pass of the same steps, kernels launched directly by "
                               "hipExtLaunchKernelGGL with start/stop HIP events on the library stream",
                  value_events_pass=round(B * args.steps / dt_events, 3), unit_launches=unit_launches)
    # the minimum bytes of the operator (coefficient once, FP64 potentials in and out per load) over the
    # whole CG iteration: how far the pass structure is from the algorithmic roofline of the matvec
    sv = survey_matvec_bytes(probs[0], 2)
    units_per_it = unit_launches / max(launches["first"], 1)
    it_gbs = units_per_it * sv / (it_ms * 1e-3) / 1e9
    common["matvec"]["algorithmic"] = dict(
        bytes_per_cell=int(sv), bytes_per_load_matvec=int(survey_matvec_bytes(probs[0], 1)),
        cells_per_iteration=round(units_per_it, 2), gbs=round(it_gbs, 1), frac=round(it_gbs / HBM_PEAK_GBS, 4),
        model="survey_matvec_bytes() in bench.py: coefficient read once per cell and iteration, FP64 potential "
              "coefficients of Z_N read and written per load; divided by the time of the whole CG iteration")
    if dom == "apply":
        # the column pass issues vector ALU work for most of its duration (its FP32
        # transforms): it is measured against the FP32 vector peak of the chip, with the
        # rate without packed FP32 instructions (which this build never emits) and its HBM view beside it
        tf = aflops / (ms * 1e-3) / 1e12
        roofline = dict(bound="alu", achieved=round(tf, 2), peak=round(VALU_PEAK_TFLOPS, 1), unit="TFLOP/s",
                        frac=round(tf / VALU_PEAK_TFLOPS, 4), peak_unpacked=round(VALU_UNPACKED_TFLOPS, 1),
                        frac_of_unpacked=round(tf / VALU_UNPACKED_TFLOPS, 4), flops_per_launch=int(aflops),
                        flops_model="apply_flops() in bench.py", hbm=hbm, **common)
    else:
        roofline = dict(bound="hbm", achieved=hbm["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=hbm["frac"],
                        bytes_per_launch=int(nbytes), **common)

    line = dict(metric=METRIC, value=round(value, 3), unit="bound pairs/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32 FFT/apply + f64 CG/bounds" if args.precision == "mixed" else "f64",
                data="synthetic",
                config=dict(workload="C2: 2D N=313 (doubled grid 625^2), random two-phase 125x125 pixel image, "
                                     "a in {1,100}, both loads, primal+dual, batched lockstep CG",
                            cells_per_step=B, tol=args.tol, precision=args.precision, cg_iters=iters,
                            solves_per_s=round(value * 2 * 2, 3),   # a bound pair: 2 primal + 2 dual load solves
                            step_ms=step_ms,
                            batched="all cells of a step in lockstep (one launch per pass covers every cell)",
                            plain_bound_pairs_per_s=None if plain_value is None else round(plain_value, 3),
                            stop=args.stop, etol=args.etol if args.stop != "residual" else None,
                            energy_rule=energy_leg, gap_rule=gap_leg, tile_tuning=tuning,
                            bound_error_vs_oracle=dict(cell=0, reference="oracle, CG to 1e-11 "
                                                                         "(tests/golden/reference_bounds.json C2)",
                                                       **(err_mixed or {})),
                            fp64=fp64_leg),
                roofline=roofline)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_cells, args.tol, results[-1])
    print(json.dumps(line), flush=True)


def _line(args, value, dt, steps, workload, extra_cfg, dtype=None):
    return dict(metric=METRIC, value=round(value, 3), unit="bound pairs/s", n_gpus=1, steps=steps,
                warmup=args.warmup, ms_per_step=round(1e3 * dt / max(steps, 1), 3), higher_is_better=True,
                scaling="weak", vs_baseline=None,
                dtype=dtype or ("f32 FFT/apply + f64 CG/bounds" if args.precision == "mixed" else "f64"),
                data="synthetic", config=dict(workload=workload, tol=args.tol, precision=args.precision,
                                              stop=args.stop, etol=args.etol if args.stop != "residual" else None,
                                              **extra_cfg),
                roofline=None)


def _c3_variant(args, anisotropic):
    """One 3D class of the C3 geometry (20 spheres, N = 41): a lockstep batch of
    args.c3_cells cells (cell 0 the configuration's own, the others new seeds),
    solved args.steps times; then the same solves with every kernel between HIP
    events for the per-pass durations."""
    import numpy as np
    import torch
    import homgen
    import paper_1404_3614_amd as H
    N = (41, 41, 41)
    name = "C3b" if anisotropic else "C3a"
    cells = [homgen.sphere_cell(1404003 + 100003 * i, n=20, anisotropic=anisotropic, rho=10.0)
             for i in range(args.c3_cells)]
    stream = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, N, precision=args.precision, stream=stream) for c in cells]
    batch = H.Batch(probs)
    rng = [H.cell_eig_range(c) for c in cells]
    batch.set_stop(args.stop, args.etol, min(r[0] for r in rng), max(r[1] for r in rng))
    for _ in range(max(1, args.warmup)):
        batch.solve_bounds(tol=args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = batch.solve_bounds(tol=args.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    batch.set_timing(True)
    for _ in range(args.steps):
        batch.solve_bounds(tol=args.tol)
    torch.cuda.synchronize()
    avg_ms, launches = batch.get_timing()
    batch.set_timing(False)
    # unit-launches per side (the 3D dual moves two components per load in the row passes)
    ul = {key: args.steps * sum(max(i["iters"] for i in cell[key]) + 1 for cell in res)
          for key in ("info_primal", "info_dual")}
    unit_launches = ul["info_primal"] + ul["info_dual"]
    plane = launches["mid_inv"] == 0        # the plane pass ran in place of the middle and column passes
    pb_p, pb_d = pass_bytes(probs[0], 3, plane, 1), pass_bytes(probs[0], 3, plane, 2)
    per_pass = {}
    for k in ("first", "mid_inv", "apply", "mid_fwd", "last"):
        if launches[k]:
            b = (ul["info_primal"] * pb_p[k] + ul["info_dual"] * pb_d[k]) / launches[k]
            per_pass[k] = dict(ms_per_launch=round(avg_ms[k], 5), bytes_per_launch=int(b),
                               gbs=round(b / (avg_ms[k] * 1e-3) / 1e9, 1), launches=launches[k])
    if plane and "apply" in per_pass:
        fl = unit_launches * plane_flops(probs[0], 3) / launches["apply"]
        per_pass["apply"].update(flops_per_launch=int(fl), tflops=round(fl / (avg_ms["apply"] * 1e-3) / 1e12, 2))
    dom = max(per_pass, key=lambda k: per_pass[k]["ms_per_launch"] * per_pass[k]["launches"])
    iters = [[i["iters"] for i in cell["info_primal"] + cell["info_dual"]] for cell in res]
    ref = golden(name)
    return dict(variant=name, cells=args.c3_cells, coefficient="10 I in I" if not anisotropic else
                "per-sphere SPD, eigenvalues log-uniform in [0.1, 10]",
                bound_pairs_per_s=round(args.c3_cells * args.steps / dt, 3), ms_per_step=round(1e3 * dt / args.steps, 3),
                cg_iters_cell0=iters[0], cg_iters_max=int(np.max(iters)),
                bound_error_vs_oracle=dict(cell=0, reference=f"oracle, CG to 1e-11 (tests/golden/reference_bounds.json "
                                                              f"{name})", **(bound_error(res[0], ref) or {})),
                per_pass=per_pass, dominant=dom, plane_pass=plane)


def run_c3(args):
    """C3: the 3D hot path on its own, lockstep batches of the configuration's
    sphere geometry (isotropic C3a, the value; anisotropic C3b beside it); the
    roofline of the dominant pass of C3a (HBM-bound: every 3D pass streams the
    doubled-grid intermediate)."""
    out = {}
    for aniso in {"both": (False, True), "a": (False,), "b": (True,)}[args.c3_variant]:
        r = _c3_variant(args, aniso)
        out[r["variant"]] = r
        print(f"[c3] {r['variant']}: {r['bound_pairs_per_s']} bound pairs/s, iterations of cell 0 {r['cg_iters_cell0']}, "
              f"bound error vs oracle {r['bound_error_vs_oracle']}", file=sys.stderr, flush=True)
    a = out.get("C3a") or out["C3b"]
    dom = a["dominant"]
    pp = a["per_pass"][dom]
    line = _line(args, a["bound_pairs_per_s"], a["ms_per_step"] * 1e-3 * args.steps, args.steps,
                 "C3: 3D N=41 (doubled grid 81^3), 20 random spheres, 3 loads, primal+dual, lockstep batch of "
                 f"{args.c3_cells} cells (" + {"both": "C3a 10 I inclusions, the value; C3b anisotropic SPD beside it",
                                              "a": "C3a 10 I inclusions",
                                              "b": "C3b anisotropic SPD inclusions"}[args.c3_variant] + ")",
                 dict(variants=out))
    names = dict(first="k_first_fast (row pass of the last axis)", mid_inv="k_mid_fast (middle axis, inverse)",
                 apply="k_plane_fast (plane pass: axes 1 and 0 inverse, coefficient, axes 0 and 1 forward)"
                 if a["plane_pass"] else "k_apply_fast (column pass: inverse FFT, coefficient, forward FFT)",
                 mid_fwd="k_mid_fast (middle axis, forward)", last="k_last_fast (row pass of the last axis)")
    hbm = dict(achieved=pp["gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=round(pp["gbs"] / HBM_PEAK_GBS, 4),
               bytes_per_launch=pp["bytes_per_launch"])
    if "tflops" in pp:
        # the plane pass moves 12.9 MB per cell but executes its FFTs from LDS: bound by vector issue
        tf = pp["tflops"]
        roof = dict(bound="alu", achieved=tf, peak=round(VALU_PEAK_TFLOPS, 1), unit="TFLOP/s",
                    frac=round(tf / VALU_PEAK_TFLOPS, 4), peak_unpacked=round(VALU_UNPACKED_TFLOPS, 1),
                    frac_of_unpacked=round(tf / VALU_UNPACKED_TFLOPS, 4), hbm=hbm,
                    flops_model="plane_flops() in bench.py (pruned line transforms as executed)")
    else:
        roof = dict(bound="hbm", **hbm)
    line["roofline"] = dict(**roof, traffic=None, kernel=f"{names[dom]} of {a['variant']}", ms_per_launch=pp["ms_per_launch"],
                            per_pass=a["per_pass"],
                            bytes_model="pass_bytes() in bench.py (primal and dual launches each with their own "
                                        "components per load); units per launch = active cells of the batch",
                            timed_region="a second run of the same solves, kernels launched directly by "
                                         "hipExtLaunchKernelGGL with start/stop HIP events on the library stream")
    print(json.dumps(line), flush=True)


def run_c4(args):
    """Mixed batch: 512 2D cells, N uniform in {13, 41, 63, 313}, and 64 3D cells at N = 41."""
    import numpy as np
    import torch
    import homgen
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd.mixed import MixedSolver
    specs = homgen.batch_specs()
    rng = [H.cell_eig_range(c) for _, c, _ in specs]
    stop_kw = dict(precision=args.precision, stop=args.stop, etol=args.theta if args.stop == "gap" else args.etol,
                   a_min=min(r[0] for r in rng), a_max=max(r[1] for r in rng))
    ms = MixedSolver(mode=args.c4_mode, **stop_kw)
    groups = ms.prepare([(N, c) for N, c, _ in specs])   # Fourier data on the device, before the timed region
    for _ in range(args.warmup):
        ms.solve(groups, len(specs), tol=args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timings = {}
    for _ in range(args.steps):
        res = ms.solve(groups, len(specs), tol=args.tol, timings=timings)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the other launch modes on the same cells, for comparison
    other_modes = {}
    for other in ("graph", "streams", "threads"):
        if other == args.c4_mode:
            continue
        ms2 = MixedSolver(mode=other, **stop_kw)
        groups2 = ms2.prepare([(N, c) for N, c, _ in specs])
        ms2.solve(groups2, len(specs), tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ms2.solve(groups2, len(specs), tol=args.tol)
        torch.cuda.synchronize()
        other_modes[other] = round(len(specs) * args.steps / (time.perf_counter() - t0), 3)
        del ms2, groups2
    classes = []
    for key, items in groups.items():
        its = np.array([[i["iters"] for i in res[j]["info_primal"] + res[j]["info_dual"]] for j, _, _ in items])
        classes.append(dict(d=key[0], N=key[1][0], cells=len(items), mean_iters=round(float(its.mean()), 1),
                            max_iters=int(its.max()), wall_ms_last_step=round(1e3 * timings[key], 2)))
    line = _line(args, len(specs) * args.steps / dt, dt, args.steps,
                 "C4: 512 2D cells (random squares, N in {13,41,63,313}) + 64 3D cells (random spheres, N=41), "
                 "contrast log-uniform in [2,1e3], d loads, primal+dual; one lockstep batch per size class, "
                 "classes concurrent on their own streams",
                 dict(cells_per_step=len(specs), classes=classes, mode=args.c4_mode,
                      other_modes=other_modes))
    # bound error of the sampled cells (the highest-contrast cell of every class) against the oracle
    sample_err = {}
    for name in ("C4s_2d_N13", "C4s_2d_N41", "C4s_2d_N63", "C4s_2d_N313", "C4s_3d_N41"):
        idx = golden_index(name)
        if idx is not None:
            sample_err[name] = dict(cell=idx, **bound_error(res[idx], golden(name)))
    line["config"]["bound_error_vs_oracle"] = sample_err
    line["roofline"] = mixed_roofline(args, ms, groups, len(specs))
    print(json.dumps(line), flush=True)


def golden_index(name):
    try:
        with open(GOLDEN) as f:
            return int(json.load(f)[name]["batch_index"])
    except (OSError, KeyError, ValueError):
        return None


def mixed_roofline(args, ms, groups, n_total):
    """Roofline of the dominant kernel of a mixed batch: every class solved once more,
    class after class with each kernel between HIP events; the (class, pass) with the
    largest total time is the dominant kernel; its algorithmic bytes (and FP32 flops
    for a column pass) per launch over its average duration."""
    res, timing = ms.solve_timed(groups, n_total, tol=args.tol)
    best, rows = None, []
    for key, items in groups.items():
        avg, cnt = timing[key]
        pb = ms.classes[key]["probs"][0]
        d = key[0]
        # a cell takes part in the launches of a solve until all its loads stopped
        uside = {k: sum(max(i["iters"] for i in res[j][k]) + 1 for j, _, _ in items)
                 for k in ("info_primal", "info_dual")}
        units = uside["info_primal"] + uside["info_dual"]
        plane = d == 3 and cnt.get("mid_inv", 0) == 0
        pb_p, pb_d = pass_bytes(pb, d, plane, 1), pass_bytes(pb, d, plane, d - 1)
        for p, c in cnt.items():
            if not c:
                continue
            tot = avg[p] * c
            b = (uside["info_primal"] * pb_p[p] + uside["info_dual"] * pb_d[p]) / c
            row = dict(cls=f"{d}D N={key[1][0]}", kernel_pass=p, ms_per_launch=round(avg[p], 5), launches=c,
                       total_ms=round(tot, 2), bytes_per_launch=int(b), gbs=round(b / (avg[p] * 1e-3) / 1e9, 1))
            if p == "apply" and args.precision == "mixed" and 2 * key[1][0] - 1 in SPLIT:
                fl = units * (plane_flops(pb, d) if plane else apply_flops(pb, d)) / c
                row.update(flops_per_launch=int(fl), tflops=round(fl / (avg[p] * 1e-3) / 1e12, 2))
            rows.append(row)
            if best is None or tot > best["total_ms"]:
                best = row
    rows.sort(key=lambda r: -r["total_ms"])
    hbm = dict(achieved=best["gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=round(best["gbs"] / HBM_PEAK_GBS, 4),
               bytes_per_launch=best["bytes_per_launch"])
    common = dict(kernel=f"{best['kernel_pass']} pass of the {best['cls']} class", ms_per_launch=best["ms_per_launch"],
                  traffic=None, per_kernel=rows[:8], bytes_model="pass_bytes() in bench.py",
                  timed_region="classes solved once more one after another, each kernel launched directly "
                               "between HIP events on its class stream")
    if "tflops" in best:
        tf = best["tflops"]
        return dict(bound="alu", achieved=tf, peak=round(VALU_PEAK_TFLOPS, 1), unit="TFLOP/s",
                    frac=round(tf / VALU_PEAK_TFLOPS, 4), peak_unpacked=round(VALU_UNPACKED_TFLOPS, 1),
                    frac_of_unpacked=round(tf / VALU_UNPACKED_TFLOPS, 4), hbm=hbm, **common)
    return dict(bound="hbm", achieved=hbm["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=hbm["frac"],
                bytes_per_launch=hbm["bytes_per_launch"], **common)


def unet_flops(d, size, levels, base, cin, cout):
    """Flops of one U-Net forward pass of one sample (2 per multiply-add of every
    convolution at its level's size; pooling, upsampling and bias not counted)."""
    import math
    import numpy as np
    from paper_1404_3614_amd import learned as LL
    sz = [list(size)]
    for _ in range(1, levels):
        sz.append([math.ceil(x / 2) for x in sz[-1]])
    pl = [int(np.prod(x)) for x in sz]
    lv = [l for l in range(levels) for _ in range(2)] + [l for l in range(levels - 2, -1, -1) for _ in range(3)] + [0]
    return sum(2 * ci * co * ks ** d * pl[l] for (ci, co, ks), l in zip(LL.layer_shapes(d, levels, base, cin, cout), lv))


def _c5_class(args, d, N, train_cells, test_cells, net_batch, steps, targets, lr, warmup):
    """Train the surrogate of one size class on solver fields, then time plain and
    learned + batched solves of the held-out cells under the three stopping rules."""
    import ctypes as C
    import numpy as np
    import torch
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib as L
    from paper_1404_3614_amd import learned as LL
    M = tuple(2 * n - 1 for n in N)
    t0 = time.perf_counter()
    X, Y, W, it_train = LL.solver_samples(train_cells, N, tol=args.tol, chunk=256 if d == 2 else 64,
                                          targets=targets)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    print(f"[c5] {d}D: {len(train_cells)} training fields in {t_gen:.1f} s", file=sys.stderr, flush=True)
    net = LL.UNet(d, M, levels=4, base=32, batch=net_batch)
    net.init_params(seed=1)
    geo = None
    if targets == "spectra":
        st = torch.cuda.Stream()
        geo = H.Batch([H.problem_from_cell(c, N, precision=args.precision, stream=st)
                       for c in train_cells[:net_batch]])
    t0 = time.perf_counter()
    hist = LL.train(net, X, Y, steps=steps, lr=lr, lr_final=lr / 20, seed=3, log_every=max(1, steps // 5), geo=geo,
                    warmup=warmup)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, Y, W, geo
    torch.cuda.empty_cache()
    st = torch.cuda.Stream()
    probs = [H.problem_from_cell(c, N, precision=args.precision, stream=st) for c in test_cells]
    batch = H.Batch(probs)
    rng = [H.cell_eig_range(c) for c in test_cells]
    a_min, a_max = min(r[0] for r in rng), max(r[1] for r in rng)
    zero = batch.bounds([[p.new_field(False) for _ in range(d)] for p in probs],
                        [[p.new_field(True) for _ in range(d)] for p in probs])
    n = len(test_cells)
    # inference alone (the network's inputs, forward passes from the captured graph, projection)
    LL.predict_x0(net, batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0p, x0d = LL.predict_x0(net, batch)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    start = batch.bounds(x0p, x0d)
    # the forward passes alone, with events on the network's stream (the inputs of every
    # test cell are written, the first net.batch of them run)
    Xall = torch.zeros((max(n, net.batch), 2) + M, dtype=torch.float32, device="cuda")
    batch.net_input(Xall)
    Xin = Xall[:net.batch]
    net.forward(Xin)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10 if d == 2 else 3
    torch.cuda.synchronize()
    e0.record(net.stream)
    for _ in range(reps):
        L.check(L.load().hom_unet_forward(net.h, C.c_void_p(Xin.data_ptr()), None), "hom_unet_forward")
    e1.record(net.stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    fwd_flops = unet_flops(d, M, 4, 32, 2, net.cout) * net.batch
    rules = {}
    for rule, etol in (("residual", None), ("guaranteed", args.etol), ("gap", args.theta)):
        batch.set_stop(rule, etol, a_min, a_max)
        tol = args.tol if rule == "residual" else 1e-12
        for _ in range(max(1, args.warmup)):
            batch.solve_bounds(tol=tol)
            x0p, x0d = LL.predict_x0(net, batch)
            batch.solve_bounds(tol=tol, x0_primal=x0p, x0_dual=x0d)
        # each solve timed on its own between synchronisations, the median taken: a solve of
        # a few milliseconds is otherwise at the mercy of one host-side stall
        reps = max(args.steps, 5)
        tp, tl = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plain = batch.solve_bounds(tol=tol)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x0p, x0d = LL.predict_x0(net, batch)
            learned = batch.solve_bounds(tol=tol, x0_primal=x0p, x0_dual=x0d)
            torch.cuda.synchronize()
            tl.append(time.perf_counter() - t0)
        t_plain, t_learned = float(np.median(tp)), float(np.median(tl))
        itp = np.array([[i["iters"] for i in b["info_primal"] + b["info_dual"]] for b in plain])
        itl = np.array([[i["iters"] for i in b["info_primal"] + b["info_dual"]] for b in learned])
        diff = max(max(float(np.abs(b1[k] - b0[k]).max() / np.linalg.norm(b0[k], 2)) for k in ("A_up", "A_low"))
                   for b0, b1 in zip(plain, learned))
        rules[rule] = dict(etol=etol, plain_batched_bound_pairs_per_s=round(n / t_plain, 2),
                           learned_batched_bound_pairs_per_s=round(n / t_learned, 2),
                           iterations_plain_mean=round(float(itp.mean()), 2),
                           iterations_plain_p95=float(np.percentile(itp, 95)),
                           iterations_learned_mean=round(float(itl.mean()), 2),
                           iterations_learned_p95=float(np.percentile(itl, 95)),
                           max_rel_bound_diff_learned_vs_plain=diff)
    batch.set_stop("residual")
    ref = batch.solve_bounds(tol=args.tol)
    ep = float(np.mean([(np.diag(s_["A_up"]) - np.diag(r["A_up"])) / (np.diag(z["A_up"]) - np.diag(r["A_up"]))
                        for s_, r, z in zip(start, ref, zero)]))
    ed = float(np.mean([(np.diag(s_["B_up"]) - np.diag(r["B_up"])) / (np.diag(z["B_up"]) - np.diag(r["B_up"]))
                        for s_, r, z in zip(start, ref, zero)]))
    return dict(d=d, N=N[0], train_cells=len(train_cells), test_cells=n,
                field_generation_s=round(t_gen, 2), adam_steps=steps, net_batch=net_batch, lr=lr, warmup=warmup,
                train_s=round(t_train, 2), loss_first=round(float(np.mean(hist[:10])), 5),
                loss_last=round(float(np.mean(hist[-max(1, steps // 20):])), 5),
                inference_and_projection_ms=round(1e3 * t_infer, 2),
                start_energy_error_vs_zero_start=dict(primal=round(ep, 4), dual=round(ed, 4)),
                forward=dict(ms_per_launch=round(fwd_ms, 4), flops_per_launch=int(fwd_flops),
                             tflops=round(fwd_flops / (fwd_ms * 1e-3) / 1e12, 2)),
                rules=rules)


def run_c5(args):
    """Learned initial guess: 4-level, 32-channel U-Nets trained on solver fields of
    2D N = 63 cells and of 3D N = 41 cells; plain versus learned + batched CG on
    held-out cells of contrast 1e2 - 1e3 under the residual, guaranteed-energy and
    gap rules, inference and projection inside the timed region."""
    import math
    import homgen
    logrho = (math.log10(2.0), 3.0)
    out = {}
    if args.c5_train > 0:
        train = [homgen.random_squares_cell(5_000_000 + i, logrho=logrho)[0] for i in range(args.c5_train)]
        test = [homgen.random_squares_cell(6_000_000 + i, logrho=(2.0, 3.0))[0] for i in range(args.c5_test)]
        out["2d"] = _c5_class(args, 2, (63, 63), train, test, 16, args.c5_steps, "grid", 2e-3, 0)
    if args.c5_train3d > 0:
        train = [homgen.random_spheres_cell(5_500_000 + i, logrho=logrho)[0] for i in range(args.c5_train3d)]
        test = [homgen.random_spheres_cell(6_500_000 + i, logrho=(2.0, 3.0))[0] for i in range(args.c5_test3d)]
        # the 3D layers have 3x the fan-in of the 2D ones: a smaller step and a warm-up keep Adam's
        # first, sign-like steps from blowing the activations up
        out["3d"] = _c5_class(args, 3, (41, 41, 41), train, test, 2, args.c5_steps3d, "spectra", 5e-4,
                              max(1, args.c5_steps3d // 10))
    main = out.get("2d") or out["3d"]
    r = main["rules"]["residual"]
    value = r["learned_batched_bound_pairs_per_s"]
    line = _line(args, value, main["test_cells"] / value * args.steps, args.steps,
                 "C5: learned + batched CG, 2D N=63 (doubled grid 125^2) random squares and 3D N=41 (81^3) random "
                 "spheres, contrast 1e2-1e3; U-Net 4 levels x 32 base channels (FP32, MFMA implicit-GEMM "
                 "convolutions) trained on solver fields",
                 dict(classes=out, value_is="2D class, residual rule, learned + batched",
                      timing="per rule: median over max(steps, 5) solves of all held-out cells, each timed "
                             "between synchronisations (learned: inference, projection and solve)"),
                 dtype="f32 FFT/apply + f64 CG/bounds; f32 network")
    fw = main["forward"]
    line["roofline"] = dict(bound="mfma", achieved=fw["tflops"], peak=157.3, unit="TFLOP/s",
                            frac=round(fw["tflops"] / 157.3, 4), traffic=None,
                            kernel="U-Net forward (implicit-GEMM convolutions on v_mfma_f32_16x16x4f32, pooling, "
                                   "upsampling), whole network per launch of net_batch samples",
                            ms_per_launch=fw["ms_per_launch"], flops_per_launch=fw["flops_per_launch"],
                            flops_model="unet_flops() in bench.py: 2 per multiply-add of every convolution",
                            timed_region="hom_unet_forward replays on the network stream between HIP events")
    print(json.dumps(line), flush=True)


def smooth_odd_at_least(n):
    """Smallest odd m >= n with no prime factors but 3 and 5."""
    m = n if n % 2 else n + 1
    while True:
        v = m
        for p in (3, 5):
            while v % p == 0:
                v //= p
        if v == 1:
            return m
        m += 2


def _ga_and_gani(H, cell, n, M, grid=None, closed=False):
    """One grid of the paper's square experiments: the Ga bounds on Z_n and the
    paper's Algorithm on the GaNi grid `grid` (n, or the even n + 1), FP64,
    residual rule 1e-8; each timed after a warm-up solve."""
    import numpy as np
    import torch
    pb = H.problem_from_cell(cell, (n, n), precision="fp64", M=(M, M))
    pb.solve_bounds(tol=1e-8)                      # warm-up: graphs, plans
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ga = pb.solve_bounds(tol=1e-8)
    torch.cuda.synchronize()
    t_ga = time.perf_counter() - t0
    pb.set_gani_from_cell(cell, grid=grid, closed=closed)
    pb.solve_bounds(tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gn = pb.solve_bounds(tol=1e-8)
    AHN, BHN = pb.gani_matrices(gn["fields_primal"], gn["fields_dual"])
    torch.cuda.synchronize()
    t_gn = time.perf_counter() - t0
    dual_start = None
    if grid is None:
        # odd grids: the dual minimisers from the primal ones (Proposition FD_odd_problem (ii) and the
        # remark on avoiding the dual solution): primal solves, A_{H,N}, the dual start, a check solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xp, _ = pb.solve(False, tol=1e-8)
        AHNp, _ = pb.gani_matrices(xp)
        x0 = pb.dual_start(xp, AHNp)
        xd, idl = pb.solve(True, x0=x0, tol=1e-8)
        b = pb.bounds(primal=xp, dual=xd)
        torch.cuda.synchronize()
        dual_start = dict(ms=round(1e3 * (time.perf_counter() - t0), 2), dual_iters=[i["iters"] for i in idl],
                          A_up=b["A_up"][0, 0], A_low=b["A_low"][0, 0])
    del pb
    it = lambda r: [i["iters"] for i in r["info_primal"] + r["info_dual"]]
    row = dict(Ga=dict(A_up=ga["A_up"][0, 0], A_low=ga["A_low"][0, 0], D=ga["D"][0, 0], iters=it(ga),
                       ms=round(1e3 * t_ga, 2)),
               GaNi=dict(A_HN=AHN[0, 0], inv_B_HN=float(np.linalg.inv(BHN)[0, 0]), A_up=gn["A_up"][0, 0],
                         A_low=gn["A_low"][0, 0], D=gn["D"][0, 0], iters=it(gn), ms=round(1e3 * t_gn, 2)))
    if dual_start is not None:
        row["GaNi_dual_from_primal"] = dual_start
    return row, t_ga + t_gn


def _square_cell(half, rho):
    import numpy as np
    import homgen
    cell = homgen.Inclusions(d=2, Y=np.array([2.0, 2.0]), A0=np.eye(2))
    cell.add("rect", [0.0, 0.0], [2 * half, 2 * half], (1.0 + rho) * np.eye(2))
    return cell


def run_e1(args):
    """The paper's odd-grid experiment: cell (-1, 1)^2, square inclusion
    |x_a| < 3/5 of coefficient (1 + rho) I in I, rho in {10, 1e3}, N = 5 3^j.
    For every grid: the Galerkin scheme with exact integration (Ga) and the
    paper's Algorithm (GaNi solve, exact bounds of its minimisers), FP64, the
    residual rule at 1e-8 of the paper's Convergence-criteria remark."""
    import paper_1404_3614_amd as H
    rows = []
    t_all = 0.0
    pairs = 0
    for rho in (10.0, 1e3):
        cell = _square_cell(0.6, rho)
        for j in range(args.e1_jmax + 1):
            n = 5 * 3 ** j
            M = smooth_odd_at_least(2 * n - 1)
            row, dt = _ga_and_gani(H, cell, n, M)
            t_all += dt
            pairs += 2
            rows.append(dict(rho=rho, N=n, M=M, **row))
            ga, gn = row["Ga"], row["GaNi"]
            dfp = row["GaNi_dual_from_primal"]
            print(f"[e1] rho {rho:g} N {n} M {M}: Ga [{ga['A_low']:.6f}, {ga['A_up']:.6f}] "
                  f"GaNi A_HN {gn['A_HN']:.6f} [{gn['A_low']:.6f}, {gn['A_up']:.6f}] "
                  f"({ga['ms']:.1f} / {gn['ms']:.1f} ms); dual from the primal: {dfp['ms']:.1f} ms, "
                  f"dual iterations {dfp['dual_iters']} instead of {gn['iters'][2:]}", file=sys.stderr, flush=True)
    line = _line(args, pairs / t_all, t_all, 1,
                 "E1: cell (-1,1)^2, square |x_a| < 3/5 of (1 + rho) I in I, rho in {10, 1e3}, N = 5 3^j, "
                 "Ga and GaNi (the paper's Algorithm) on each grid, FP64, residual rule 1e-8",
                 dict(grids=rows), dtype="f64")
    line["config"]["tol"] = 1e-8
    line["config"]["precision"] = "fp64"
    print(json.dumps(line), flush=True)


def run_e2(args):
    """The paper's even-grid experiment: cell (-1, 1)^2, the open square
    |x_a| < 3/4 (S1) and the closed square |x_a| <= 3/4 (S2) of coefficient
    (1 + rho) I in I, rho in {10, 1e3}, GaNi grids n = 2^j.  The GaNi fields
    are the trigonometric polynomials of the reduced set, Z_{n-1}; per grid:
    A_{H,N}, B_{H,N}^-1 (a duality gap on even grids), the exact bounds of the
    minimisers, and the Ga bounds on the same space Z_{n-1}.  FP64, residual
    rule 1e-8."""
    import paper_1404_3614_amd as H
    rows = []
    t_all = 0.0
    pairs = 0
    for topo, closed in (("S1", False), ("S2", True)):
        for rho in (10.0, 1e3):
            cell = _square_cell(0.75, rho)
            for j in range(2, args.e2_jmax + 1):
                g = 2 ** j
                n = g - 1
                M = smooth_odd_at_least(2 * n - 1)
                row, dt = _ga_and_gani(H, cell, n, M, grid=(g, g), closed=closed)
                t_all += dt
                pairs += 2
                rows.append(dict(cell=topo, rho=rho, grid=g, N=n, M=M, **row))
                ga, gn = row["Ga"], row["GaNi"]
                print(f"[e2] {topo} rho {rho:g} grid {g} (fields {n}, M {M}): GaNi A_HN {gn['A_HN']:.6f} "
                      f"B_HN^-1 {gn['inv_B_HN']:.6f} bounds [{gn['A_low']:.6f}, {gn['A_up']:.6f}]; "
                      f"Ga [{ga['A_low']:.6f}, {ga['A_up']:.6f}] ({ga['ms']:.1f} / {gn['ms']:.1f} ms)",
                      file=sys.stderr, flush=True)
    line = _line(args, pairs / t_all, t_all, 1,
                 "E2: cell (-1,1)^2, open square |x_a| < 3/4 (S1) and closed |x_a| <= 3/4 (S2) of (1 + rho) I in I, "
                 "rho in {10, 1e3}, GaNi on even grids n = 2^j (fields on Z_{n-1}) and Ga on Z_{n-1}, FP64, "
                 "residual rule 1e-8", dict(grids=rows), dtype="f64")
    line["config"]["tol"] = 1e-8
    line["config"]["precision"] = "fp64"
    print(json.dumps(line), flush=True)


def run_e3(args):
    """The paper's foam example at its size, on a synthetic stand-in image: a
    1200 x 1200 two-phase pixel image (fly ash 0.49 with overlapping circular
    air pores 0.029, pore fraction 0.5, seeded), GaNi on the even grid 1200
    (fields on Z_1199) and the Ga bounds of Z_1199 (quadrature grid 3125), for
    the original and the smoothed image; FP64, residual rule 1e-8.  The paper
    reports about fifteen minutes for GaNi and the bounds of its 1200^2 image on
    a two-core laptop CPU."""
    import numpy as np
    import torch
    import homgen
    import paper_1404_3614_amd as H
    cell0 = homgen.foam_cell(1404008, P=1200)
    rows = []
    t_all = 0.0
    pairs = 0
    for name, cell in (("original", cell0), ("smoothed", H.smooth_pixel_cell(cell0))):
        n, g, M = 1199, 1200, 3125
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb = H.problem_from_cell(cell, (n, n), precision="fp64", M=(M, M))
        ga = pb.solve_bounds(tol=1e-8)
        torch.cuda.synchronize()
        t_ga = time.perf_counter() - t0
        t0 = time.perf_counter()
        pb.set_gani_from_cell(cell, grid=(g, g))
        gn = pb.solve_bounds(tol=1e-8)
        AHN, BHN = pb.gani_matrices(gn["fields_primal"], gn["fields_dual"])
        torch.cuda.synchronize()
        t_gn = time.perf_counter() - t0
        del pb
        t_all += t_ga + t_gn
        pairs += 2
        it = lambda r: [i["iters"] for i in r["info_primal"] + r["info_dual"]]
        rows.append(dict(image=name, grid=g, N=n, M=M,
                         GaNi=dict(A_HN=AHN.tolist(), inv_B_HN=np.linalg.inv(BHN).tolist(), A_up=gn["A_up"].tolist(),
                                   A_low=gn["A_low"].tolist(), D=gn["D"].tolist(), iters=it(gn),
                                   s=round(t_gn, 3)),
                         Ga=dict(A_up=ga["A_up"].tolist(), A_low=ga["A_low"].tolist(), D=ga["D"].tolist(),
                                 iters=it(ga), s=round(t_ga, 3))))
        print(f"[e3] {name}: GaNi A_HN {AHN[0, 0]:.7f} {AHN[1, 1]:.7f} B_HN^-1 {np.linalg.inv(BHN)[0, 0]:.7f}; "
              f"bounds [{gn['A_low'][0, 0]:.7f}, {gn['A_up'][0, 0]:.7f}] ({t_gn:.2f} s); Ga bounds "
              f"[{ga['A_low'][0, 0]:.7f}, {ga['A_up'][0, 0]:.7f}] ({t_ga:.2f} s, set-up included)",
              file=sys.stderr, flush=True)
    line = _line(args, pairs / t_all, t_all, 1,
                 "E3: synthetic stand-in for the paper's 1200^2 foam image (ash 0.49, air pores 0.029, pore fraction "
                 "0.5), GaNi on the grid 1200 and Ga on Z_1199 (M 3125), original and smoothed, FP64, residual 1e-8",
                 dict(images=rows, paper_context="about 15 min for GaNi and bounds of the 1200^2 image on an Intel "
                                                 "Core i5-4200M (2 cores, 2.5 GHz), 8 GB"), dtype="f64")
    line["config"]["tol"] = 1e-8
    line["config"]["precision"] = "fp64"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
