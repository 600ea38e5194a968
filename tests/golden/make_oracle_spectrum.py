"""Write the oracle's eigenvalues of the D-N iteration matrix (tests/golden/oracle_spectrum_h16.json).

    OMP_NUM_THREADS=8 python tests/golden/make_oracle_spectrum.py   (about 15 minutes on 8 cores)

Calls only the oracle (``oracle/``) and the surface generator (``workloads/``):
the dense matrix of eq. (A_mat), section "Discrete iteration operator", on the
unit sphere at h = 1/16 (N = 4302, delta = 3h, mu = 1, gamma = 0), built from
the oracle's dense layer matrices, and its eigenvalues by LAPACK.  The
configurations of the paper's figure of these eigenvalues: kappa = 1 with
theta = 0.5 and 0.75; kappa = 1e-2 and 1e-4 with theta = c kappa, c = 0.5,
0.75, 0.9.  Stored per configuration: the 60 eigenvalues farthest from
1 - theta (where the high harmonics cluster), in that order.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workloads import surfaces  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_spectrum_h16.json")
CONFIGS = [(1.0, 0.5), (1.0, 0.75)] + [(K, c * K) for K in (1e-2, 1e-4) for c in (0.5, 0.75, 0.9)]


def main() -> int:
    h = 1.0 / 16
    S = surfaces.sphere(h)
    geo = O.Geometry(S.x, S.n, S.w, 3 * h)
    out = {"_source": "oracle.dn_iteration_eigenvalues on the unit sphere, h = 1/16 (N = %d), delta = 3h, mu = 1, "
                      "gamma = 0: eq. (A_mat), section 'Discrete iteration operator'; the 60 eigenvalues farthest "
                      "from 1 - theta, in that order; written by tests/golden/make_oracle_spectrum.py" % S.N,
           "configs": []}
    for K, theta in CONFIGS:
        t0 = time.perf_counter()
        lam = O.dn_iteration_eigenvalues(geo, 1.0, K, theta, k=60)
        print(f"K={K:g} theta={theta:g}: {lam[:4]} ... {time.perf_counter() - t0:.0f} s", flush=True)
        out["configs"].append({"K": K, "theta": theta, "re": [float(v.real) for v in lam],
                               "im": [float(v.imag) for v in lam]})
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
