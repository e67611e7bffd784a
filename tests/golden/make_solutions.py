"""Writes tests/golden/<workload>_oracle.npz: the FP64 oracle's solution of
workloads whose oracle solve takes minutes (the Huber generator at
F 10000 x 4000, 40 entries per row), so that device solves of the same
instance can be compared with it in seconds.  Calls only the oracle and the
input generators.

Stored: x (the primal solution), pobj (objective), iters, and the final
pres, dres, gap of the oracle's own stopping test.

usage: python tests/golden/make_solutions.py [workload ...]
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import ipm  # noqa: E402
from synth import problems  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def path(name):
    return os.path.join(HERE, f"{name}_oracle.npz")


def write(name):
    prob = problems.workload(name)
    t = time.time()
    r = ipm.solve(prob)
    assert r.status == ipm.SOLVED, r.status
    np.savez_compressed(path(name), x=r.x, pobj=r.pobj, iters=r.iters, pres=r.pres, dres=r.dres, gap=r.gap,
                        n=prob.n, m=prob.m, p=prob.p)
    return time.time() - t, r


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["huber_s"]:
        dt, r = write(nm)
        print(nm, f"{dt:.1f} s", "iters", r.iters, "pobj", r.pobj, flush=True)
