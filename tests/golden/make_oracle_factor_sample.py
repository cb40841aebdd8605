"""Writes a fixed sample of the FP64 oracle's factor of a named workload to
tests/golden/.

The 64^3 7-point Laplacian's factor (156,651,713 entries) takes the oracle
about five minutes on one core and 1.3 GB, too much to repeat in a
test or to store, so every STRIDE-th entry of the oracle's exact structure
(column by column, rows increasing) is stored with its row, column and the
column's diagonal entry L_jj; the file is keyed by the SHA-256 of
oracle/oracle.c and of the input generator, and a reader that finds other
hashes treats it as stale.  Only the oracle (oracle/) computes what is stored.

    python tests/golden/make_oracle_factor_sample.py lap3d_7pt_64
"""
from __future__ import annotations

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
from tests.golden.make_oracle_solution import source_hashes  # noqa: E402

STRIDE = 997  # prime, so the sample walks every row offset of every column length


def path_for(name):
    return os.path.join(HERE, "oracle_L_sample_%s.npz" % name)


def load(name):
    """dict(rows, cols, vals, ljj, stride, nnz_l) of the stored sample, or None
    when absent or stale."""
    path = path_for(name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        meta = {k: str(z[k]) for k in ("oracle_sha", "inputs_sha", "workload")}
        if meta != dict(source_hashes(), workload=name):
            return None
        return {k: np.array(z[k]) for k in ("rows", "cols", "vals", "ljj", "stride", "nnz_l")}


def main(name):
    t0 = time.time()
    p = inputs.make_workload(name)
    print("workload", name, "n", p.n, "nnz", p.nnz, flush=True)
    Cp, Ci, Cx, _ = oracle.permute(p.n, p.colptr, p.rowind, p.values, p.perm)
    sym = oracle.symbolic(p.n, Cp, Ci)
    st, Lx = oracle.factor(p.n, Cp, Ci, Cx, sym)
    assert st == 0, st
    print("oracle factor done in %.0f s, nnz(L) %d" % (time.time() - t0, Lx.size), flush=True)
    q = np.arange(0, Lx.size, STRIDE, dtype=np.int64)
    cols = (np.searchsorted(sym.Lp, q, side="right") - 1).astype(np.int32)
    rows = np.asarray(sym.Li)[q].astype(np.int32)
    ljj = Lx[np.asarray(sym.Lp)[cols]]
    np.savez_compressed(path_for(name), rows=rows, cols=cols, vals=Lx[q], ljj=ljj,
                        stride=np.int64(STRIDE), nnz_l=np.int64(Lx.size),
                        workload=np.str_(name),
                        **{k: np.str_(v) for k, v in source_hashes().items()})
    print("stored %d entries" % q.size, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "lap3d_7pt_64")
