"""Write the oracle's coupled solutions at h = 1/32 (tests/golden/oracle_solves_h32.npz).

    OMP_NUM_THREADS=8 python tests/golden/make_oracle_solves.py   (about 30 minutes on 8 cores)

Calls only the oracle (``oracle/``) and the input generators (``workloads/``):
the matrix-free Dirichlet-Neumann solve of section "Algorithm" with the
interface equation solved by GMRES (outer "gmres", theta cancels), local
GMRES solves of eqs. (Darcy_final) and (Stokes_final) with implicit slip,
every pair sum an FP64 loop of ``oracle_sums.c``.  Tolerances: local 1e-12,
interface 1e-11 (relative residuals).

Cases (delta = 3h, mu = 1), the benchmark configurations at h = 1/32 that the
dense brute force cannot reach (4N = 68280 unknowns):
  sphere_K1e-2_a1    unit sphere (N = 17070), K = 1e-2, alpha = 1, U = e_z
  sphere_K1_a0.1     unit sphere, K = 1, alpha = 0.1, U = e_z
  ellipsoid_K1e-2_a1 ellipsoid x^2 + y^2/0.64 + z^2/0.36 = 1 (N = 10618),
                     K = 1e-2, alpha = 1, U = workloads.fields.unit_vector(31)
Stored per case: p [N], u [3, N], drag [3], the interface iterations, and the
parameters; the GPU test (tests/test_gpu_oracle_h32.py) compares its own FP64
and mixed solves with them element by element.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workloads import fields, surfaces  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_solves_h32.npz")

CASES = [
    ("sphere_K1e-2_a1", "sphere", 1e-2, 1.0, None),
    ("sphere_K1_a0.1", "sphere", 1.0, 0.1, None),
    ("ellipsoid_K1e-2_a1", "ellipsoid", 1e-2, 1.0, 31),
]
TOL_GMRES, TOL_DDM = 1e-12, 1e-11


def surface(kind, h):
    if kind == "sphere":
        return surfaces.sphere(h)
    return surfaces.ellipsoid(h, 1.0, 0.8, 0.6)


def main() -> int:
    h = 1.0 / 32
    out = {}
    for name, kind, K, alpha, useed in CASES:
        S = surface(kind, h)
        U = np.array([0.0, 0.0, 1.0]) if useed is None else fields.unit_vector(useed)
        geo = O.Geometry(S.x, S.n, S.w, 3 * h)
        ops = O.Operators(geo, 1.0)
        t0 = time.perf_counter()
        p, u, D, info = O.ddm_solve(ops, O.Params(1.0, K, alpha), U, None,
                                    O.Opts(tol_gmres=TOL_GMRES, tol_ddm=TOL_DDM, outer="gmres"))
        dt = time.perf_counter() - t0
        print(f"{name}: N={S.N} drag {D} interface iterations {info.ddm_iters} residual {info.ddm_res} "
              f"applies {ops.napply} {dt:.0f} s", flush=True)
        out[f"{name}/p"] = p
        out[f"{name}/u"] = u
        out[f"{name}/drag"] = D
        out[f"{name}/U"] = U
        out[f"{name}/params"] = np.array([1.0, K, alpha, 3 * h, TOL_GMRES, TOL_DDM])
        out[f"{name}/ddm_iters"] = np.array(info.ddm_iters)
        out[f"{name}/N"] = np.array(S.N)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
