"""Write tests/golden/reference_bounds.json from the FP64 oracle only.

Usage:  python -m oracle.make_golden [--only C1,C2,...]

For each configuration the oracle runs d primal and d dual CG solves to the
reference tolerance 1e-11 (relative residual, Convergence-criteria remark of
Sec. 7.2) and records the guaranteed bounds (Def. upper_lower_bounds), the
Voigt/Reuss means and the CG iteration counts needed to reach 1e-6, 1e-8 and
1e-11.  Inputs come from the seeded generators in ``homgen``.

The C4 sample ("C4s_<d>d_N<N>") is the highest-contrast cell of every size
class of the mixed batch ``homgen.batch_specs()`` (512 random-square 2D cells
with N in {13, 41, 63, 313} and 64 random-sphere 3D cells at N = 41, contrast
log-uniform in [2, 1e3]); the entry records its index in the batch.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import time

import numpy as np

import homgen
from . import galerkin as ga

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "tests", "golden", "reference_bounds.json")

CONFIGS = {
    # 2D N=13: centred square inclusion, vf 0.25, A = 10 I in A = I
    "C1": dict(cell=lambda: homgen.square_inclusion_cell(d=2, side=0.5, rho_in=10.0), N=13),
    # 2D N=313: 125x125 Bernoulli(0.5) pixel image, a in {1, 100}
    "C2": dict(cell=lambda: homgen.pixel_cell(1404002, P=125, values=(1.0, 100.0)), N=313),
    # 3D N=41: 20 non-overlapping spheres r in [0.08, 0.15], 10 I in I
    "C3a": dict(cell=lambda: homgen.sphere_cell(1404003, n=20, anisotropic=False, rho=10.0), N=41),
    # same geometry, anisotropic SPD inclusions with eigenvalues log-uniform in [0.1, 10]
    "C3b": dict(cell=lambda: homgen.sphere_cell(1404003, n=20, anisotropic=True), N=41),
}


def c4_sample():
    """{name: (index, N, cell)}: the highest-contrast cell of each size class of
    the default mixed batch."""
    pick = {}
    for i, (N, cell, rho) in enumerate(homgen.batch_specs()):
        key = (cell.d, N)
        if key not in pick or rho > pick[key][2]:
            pick[key] = (i, cell, rho)
    return {f"C4s_{d}d_N{N}": (i, N, cell, rho) for (d, N), (i, cell, rho) in sorted(pick.items())}


for _name, (_i, _N, _cell, _rho) in c4_sample().items():
    CONFIGS[_name] = dict(cell=(lambda c=_cell: c), N=_N, batch_index=_i, rho=_rho)


def first_below(hist, tol):
    for i, r in enumerate(hist):
        if r <= tol:
            return i
    return None


def run(name, spec, tol=1e-11):
    t0 = time.time()
    cell = spec["cell"]()
    prob = ga.make_problem(cell, spec["N"])
    d = prob.d
    I = np.eye(d)
    prim, dual, its = [], [], {"primal": [], "dual": []}
    for a in range(d):
        for kind, store in (("primal", prim), ("dual", dual)):
            r = ga.solve(prob, I[a], dual=(kind == "dual"), tol=tol)
            store.append(r.x)
            its[kind].append({f"{t:g}": first_below(r.res_hist, t) for t in (1e-6, 1e-8, 1e-11)})
    b = ga.bounds_from_fields(prob, prim, dual)
    voigt, reuss = ga.voigt_reuss(prob)
    out = {k: np.asarray(v).tolist() for k, v in b.items()}
    if "batch_index" in spec:
        out.update(batch_index=spec["batch_index"], rho=spec["rho"])
    out.update(d=d, N=list(prob.N), M=list(prob.M), tol=tol, iters=its,
               voigt=voigt.tolist(), reuss=reuss.tolist(), seconds=round(time.time() - t0, 2))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    names = args.only.split(",") if args.only else list(CONFIGS)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for n in names:
        print(f"[golden] {n} ...", flush=True)
        data[n] = run(n, CONFIGS[n])
        print(f"[golden] {n} done in {data[n]['seconds']} s", flush=True)
        data["_meta"] = dict(generator="python -m oracle.make_golden", numpy=np.__version__,
                             host=platform.processor() or platform.machine())
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
