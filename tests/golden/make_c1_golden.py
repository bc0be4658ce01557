"""Write ``c1_poisson31.json``: the oracle's results on the 31^3
variable-coefficient Poisson workload (lognormal kappa = exp(g), unit
variance, correlation length 0.2; f ~ U(-1, 1); eps 1e-6, eta 2, leaf 32).

Stored: sampled entries and 2-norms of
  z  = M^{-1} f   (the oracle's FP64 H-matrix cyclic reduction, Sec. 4.1-4.2),
  zt = M^{-T} f   (its exact transpose),
  x  = A^{-1} f   (sparse direct solve of the assembled operator, Sec. 6),
and the oracle's rank statistics.  Only ``oracle/`` and the seeded input
generators are used; about 1.5 minutes on one core.

    python tests/golden/make_c1_golden.py
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

NSAMPLE = 1024
SAMPLE_SEED = 7


def main():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    inp = synth.config_inputs("poisson31")
    n = inp["n"]
    N = n ** 3
    S = assembly.stencil7("poisson", n, n, n, kappa=inp["kappa"])
    t0 = time.time()
    H = hacr.HACR(S, n, n, n, eps=inp["eps"], eta=inp["eta"], leaf=inp["leaf"])
    t1 = time.time()
    f = inp["f"]
    z = H.apply(f)
    zt = H.apply_T(f)
    x = spla.spsolve(assembly.to_sparse(S, n, n, n).tocsc(), f)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(N, NSAMPLE, replace=False))
    st = H.stats()
    out = {
        "workload": "poisson31",
        "n": n, "eps": inp["eps"], "eta": inp["eta"], "leaf": inp["leaf"],
        "oracle_setup_seconds": round(t1 - t0, 1),
        "max_rank": {str(k): int(v) for k, v in st["max_rank"].items()},
        "index": idx.tolist(),
        "z": [float(v) for v in z[idx]], "z_norm": float(np.linalg.norm(z)),
        "zt": [float(v) for v in zt[idx]], "zt_norm": float(np.linalg.norm(zt)),
        "x": [float(v) for v in x[idx]], "x_norm": float(np.linalg.norm(x)),
    }
    path = os.path.join(HERE, "c1_poisson31.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {path} (oracle setup {t1 - t0:.1f} s)")


if __name__ == "__main__":
    main()
