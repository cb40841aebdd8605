"""Writes the FP64 oracle's solution of a named workload to tests/golden/.

The 27-point 3-dof 48^3 problem (n = 331,776, 8 right-hand sides) takes the
oracle about 15 minutes on one core, too long to repeat inside a test or a
benchmark run, so its solution is stored once, keyed by the SHA-256 of
oracle/oracle.c and of the input generator: a reader that finds other hashes
treats the file as stale.  Only the oracle (oracle/) computes what is stored.

    python tests/golden/make_oracle_solution.py elast27_48
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1608_00044_amd import inputs  # noqa: E402


def source_hashes():
    out = {}
    for key, path in (("oracle_sha", os.path.join(ROOT, "oracle", "oracle.c")),
                      ("inputs_sha", os.path.join(ROOT, "paper_1608_00044_amd", "inputs.py"))):
        with open(path, "rb") as f:
            out[key] = hashlib.sha256(f.read()).hexdigest()
    return out


def path_for(name):
    return os.path.join(HERE, "oracle_x_%s.npz" % name)


def load(name):
    """(x, meta) of the stored solution, or None when absent or stale."""
    path = path_for(name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        meta = {k: str(z[k]) for k in ("oracle_sha", "inputs_sha", "workload")}
        if meta != dict(source_hashes(), workload=name):
            return None
        return np.array(z["x"]), dict(meta, eta=np.array(z["eta"]), seed=int(z["seed"]))


def main(name):
    t0 = time.time()
    p = inputs.make_workload(name)
    print("workload", name, "n", p.n, "nnz", p.nnz, "rhs", p.rhs.shape[1], flush=True)
    out = oracle.run(p, ratio=0.0)
    assert out["status"] == 0, out["status"]
    x = np.asfortranarray(out["x"]).reshape(p.n, -1)
    eta = oracle.backward_error(p.n, p.colptr, p.rowind, p.values, p.rhs, x)
    print("oracle done in %.0f s, eta %s" % (time.time() - t0, eta), flush=True)
    np.savez_compressed(path_for(name), x=np.ascontiguousarray(x), eta=eta,
                        seed=np.int64(p.meta["seed"]), workload=np.str_(name),
                        **{k: np.str_(v) for k, v in source_hashes().items()})


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "elast27_48")
