"""Write ``poisson63_subcube.json``: the oracle's results on a 63^3
variable-coefficient Poisson problem with the 8^3 sub-cube kappa of six
decades (values 10^U(-3,3), seed 11; f ~ U(-1, 1), seed 12; eps 1e-4,
eta 2, leaf 32), the recipe of the 127^3 workload at the size whose planes
(3969 unknowns, 6 cyclic-reduction levels) still fit the oracle.

Stored: sampled entries and 2-norms and max-norms of
  z  = M^{-1} f   (the oracle's FP64 H-matrix cyclic reduction, Sec. 4.1-4.2),
  zt = M^{-T} f   (its exact transpose),
  x  = A^{-1} f   (sparse direct solve of the assembled operator, Sec. 6),
and the oracle's rank statistics.  Only ``oracle/`` and the seeded input
generators are used; tens of minutes on one core.

    python tests/golden/make_poisson63_golden.py
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import assembly, hacr  # noqa: E402

NSAMPLE = 2048
SAMPLE_SEED = 8


def main():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    n, eps, eta, leaf = 63, 1e-4, 2.0, 32
    N = n ** 3
    kap = synth.kappa_subcubes(n, 11)
    f = synth.rhs_uniform(N, 12)
    S = assembly.stencil7("poisson", n, n, n, kappa=kap)
    t0 = time.time()
    H = hacr.HACR(S, n, n, n, eps=eps, eta=eta, leaf=leaf)
    t1 = time.time()
    z = H.apply(f)
    zt = H.apply_T(f)
    x = spla.spsolve(assembly.to_sparse(S, n, n, n).tocsc(), f)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(N, NSAMPLE, replace=False))
    st = H.stats()
    out = {
        "workload": "poisson63_subcube",
        "n": n, "eps": eps, "eta": eta, "leaf": leaf, "kappa_seed": 11, "f_seed": 12,
        "oracle_setup_seconds": round(t1 - t0, 1),
        "max_rank": {str(k): int(v) for k, v in st["max_rank"].items()},
        "index": idx.tolist(),
        "z": [float(v) for v in z[idx]], "z_norm": float(np.linalg.norm(z)), "z_max": float(np.abs(z).max()),
        "zt": [float(v) for v in zt[idx]], "zt_norm": float(np.linalg.norm(zt)),
        "zt_max": float(np.abs(zt).max()),
        "x": [float(v) for v in x[idx]], "x_norm": float(np.linalg.norm(x)),
        "oracle_vs_exact": float(np.linalg.norm(z - x) / np.linalg.norm(x)),
    }
    path = os.path.join(HERE, "poisson63_subcube.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {path} (oracle setup {t1 - t0:.1f} s)")


if __name__ == "__main__":
    main()
