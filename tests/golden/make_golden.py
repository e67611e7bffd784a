"""Writes tests/golden/patterns.json: digests of the oracle's symbolic
analysis (permutation, etree, column counts, supernode partitions and row
lists) for the named workloads, so that the library's analysis can be
compared bit for bit at sizes where the oracle's plain ordering takes
minutes.  Calls only the oracle and the input generators.

usage: python tests/golden/make_golden.py [workload[@nd] ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import kkt, symbolic  # noqa: E402
from synth import problems  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "patterns.json")


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def pattern_record(key):
    # "name" is the minimum-degree analysis of a workload, "name@nd" its nested-dissection analysis
    name, _, ordering = key.partition("@")
    prob = problems.workload(name)
    t = time.time()
    pat = symbolic.analyze(kkt.kkt_pattern(prob), ordering or "md")
    if key in ("lasso", "huber_l"):
        # the oracle's ordering of a benchmark workload, for the CPU-baseline
        # leg of the benchmark (which then needs only the fast symbolic steps)
        np.save(os.path.join(os.path.dirname(OUT), f"{name}_perm.npy"), pat.perm.astype(np.int32))
    return dict(
        N=int(pat.N), nnz_L=int(pat.nnz_L), nsuper_fund=int(len(pat.super_fund) - 1),
        nsuper=int(len(pat.super_ptr) - 1), rows_total=int(len(pat.rows)),
        perm=digest(pat.perm, np.int32), parent=digest(pat.parent, np.int32),
        colcount=digest(pat.colcount, np.int64), super_fund=digest(pat.super_fund, np.int32),
        super_ptr=digest(pat.super_ptr, np.int32), rows_ptr=digest(pat.rows_ptr, np.int64),
        rows=digest(pat.rows, np.int32), oracle_seconds=round(time.time() - t, 1))


if __name__ == "__main__":
    names = sys.argv[1:] or ["small_qp", "lasso_s", "many_soc_s", "lasso_diff_s", "huber_s", "lasso"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        data[nm] = pattern_record(nm)
        print(nm, data[nm]["N"], data[nm]["nnz_L"], data[nm]["oracle_seconds"], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
