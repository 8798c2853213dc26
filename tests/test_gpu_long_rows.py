"""GPU: row passes for lines that do not fit in LDS.

The fused row passes hold both lines of a row pair in LDS; for long rows
(e.g. the paper's grids N = 1023 and 1215 in FP64) they run split, as the
gather (or epilogue) kernel plus a separate row transform over HBM, with the
same arithmetic per line.  HOM_LONG_ROWS forces the split form at any size:
results are bitwise those of the fused form.  At full size the Ga bounds of
nested spaces Z_511 within Z_1023 are monotone (Sec. 6: the minimisation
spaces grow), and the even-grid GaNi of the paper's squares runs on the grid
1024."""
import os
import subprocess
import sys

import numpy as np
import pytest

import homgen

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1404_3614_amd as H
    from paper_1404_3614_amd import _lib
    _lib.load()
    return H


def _square(half, rho):
    c = homgen.Inclusions(d=2, Y=np.array([2.0, 2.0]), A0=np.eye(2))
    c.add("rect", [0.0, 0.0], [2 * half, 2 * half], (1.0 + rho) * np.eye(2))
    return c


# one process per form: the switch is read at launch, graphs are cached per problem
_SCRIPT = r"""
import json, sys
import numpy as np
sys.path.insert(0, %(root)r)
sys.path.insert(0, %(tests)r)
import homgen, paper_1404_3614_amd as H
from test_gpu_long_rows import CASES
out = {}
for name, make, N, M, prec, grid in CASES:
    cell = make()
    pb = H.problem_from_cell(cell, N, precision=prec, M=M)
    r = pb.solve_bounds(tol=1e-10 if prec == "fp64" else 1e-8)
    res = dict(A_up=r["A_up"].tolist(), A_low=r["A_low"].tolist(),
               iters=[i["iters"] for i in r["info_primal"] + r["info_dual"]])
    if grid is not None:
        pb.set_gani_from_cell(cell, grid=grid, closed=True)
        g = pb.solve_bounds(tol=1e-10 if prec == "fp64" else 1e-8)
        AHN, BHN = pb.gani_matrices(g["fields_primal"], g["fields_dual"])
        res.update(G_up=g["A_up"].tolist(), G_low=g["A_low"].tolist(), AHN=AHN.tolist(), BHN=BHN.tolist())
    out[name] = res
    print("[long-rows] case", name, "done", file=sys.stderr, flush=True)
print(json.dumps(out))
"""

CASES = [
    ("sq2d_fp64", lambda: _square(0.6, 10.0), (39, 39), (81, 81), "fp64", (40, 40)),
    ("sq2d_mixed", lambda: _square(0.6, 100.0), (41, 27), (81, 75), "mixed", None),
    ("pix2d_mixed", lambda: homgen.pixel_cell(seed=3, P=25, values=(1.0, 30.0)), (41, 63), None, "mixed", None),
    ("sph3d_fp64", lambda: homgen.sphere_cell(seed=4, n=4, anisotropic=True), (5, 9, 5), (9, 25, 9), "fp64", (6, 10, 6)),
    ("sph3d_mixed", lambda: homgen.sphere_cell(seed=5, n=5, anisotropic=False), (13, 5, 13), None, "mixed", None),
]


def _run(long_rows):
    env = dict(os.environ)
    env.pop("HOM_LONG_ROWS", None)
    if long_rows:
        env["HOM_LONG_ROWS"] = "1"
    code = _SCRIPT % dict(root=ROOT, tests=os.path.join(ROOT, "tests"))
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    sys.stderr.write(p.stderr[-2000:])
    assert p.returncode == 0, p.stderr[-2000:]
    import json
    return json.loads(p.stdout.strip().splitlines()[-1])


def test_split_row_passes_are_bitwise_the_fused_ones():
    fused = _run(False)
    split = _run(True)
    for name, *_ in CASES:
        a, b = fused[name], split[name]
        print(f"[long-rows] {name}: iterations {a['iters']} / {b['iters']}", flush=True)
        assert a == b, name


def test_full_size_nested_grids_and_even_gani():
    """FP64 Ga on Z_1023 (quadrature grid 2187: rows too long for the fused
    passes) against Z_511; GaNi of the closed square on the grid 1024."""
    H = _H()
    cell = _square(0.75, 10.0)
    small = H.problem_from_cell(cell, (511, 511), precision="fp64", M=(1125, 1125)).solve_bounds(tol=1e-9)
    pb = H.problem_from_cell(cell, (1023, 1023), precision="fp64", M=(2187, 2187))
    big = pb.solve_bounds(tol=1e-9)
    n = np.linalg.norm(big["A_up"], 2)
    print(f"[long-rows] Z_511 [{small['A_low'][0, 0]:.6f}, {small['A_up'][0, 0]:.6f}] "
          f"Z_1023 [{big['A_low'][0, 0]:.6f}, {big['A_up'][0, 0]:.6f}]", flush=True)
    assert np.linalg.eigvalsh(small["A_up"] - big["A_up"]).min() >= -1e-9 * n
    assert np.linalg.eigvalsh(big["A_low"] - small["A_low"]).min() >= -1e-9 * n
    assert np.linalg.eigvalsh(big["A_up"] - big["A_low"]).min() > 0
    # the energy of the CG recurrence is the diagonal of the upper bound
    ep = np.array([i["energy"] for i in big["info_primal"]])
    assert np.abs(ep - np.diag(big["A_up"])).max() <= 1e-8 * n
    pb.set_gani_from_cell(cell, grid=(1024, 1024), closed=True)
    g = pb.solve_bounds(tol=1e-9)
    AHN, BHN = pb.gani_matrices(g["fields_primal"], g["fields_dual"])
    gap = np.linalg.eigvalsh(AHN - np.linalg.inv(BHN))
    print(f"[long-rows] GaNi grid 1024: A_HN {AHN[0, 0]:.6f} B_HN^-1 {np.linalg.inv(BHN)[0, 0]:.6f} "
          f"bounds [{g['A_low'][0, 0]:.6f}, {g['A_up'][0, 0]:.6f}]", flush=True)
    assert gap.min() >= -1e-9 * n
    # the exact bounds of any fields of Z_1023 enclose the Ga bounds of that space
    assert np.linalg.eigvalsh(g["A_up"] - big["A_up"]).min() >= -1e-9 * n
    assert np.linalg.eigvalsh(big["A_low"] - g["A_low"]).min() >= -1e-9 * n
