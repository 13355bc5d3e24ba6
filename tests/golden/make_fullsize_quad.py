"""Writes the exact (__float128) sampled outputs of the two large workloads.

    python tests/golden/make_fullsize_quad.py [gravity_1024] [magnetic_288]

For each workload it evaluates, with the CPU oracle only, single rows of G m
and single columns of G^T r at the seeded stations and prisms of
``workloads.fullsize_case`` with every corner term, entry and sum in
__float128 (``oracle.station_sums(..., quad=True)``, ``oracle.prism_sums(...,
quad=True)``), and writes them to ``fullsize_quad_<name>.txt`` beside this
script.  The values are the products' definition (Sec. 2, eq. Gslice)
evaluated exactly up to the final rounding to double.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def write(name):
    pr, m, r, st, pq = W.fullsize_case(name)
    P = oracle.problem_from_dict(pr)
    t0 = time.time()
    ds = oracle.station_sums(P, m, st, quad=True)
    ts = oracle.prism_sums(P, r, pq, quad=True)
    path = os.path.join(HERE, "fullsize_quad_%s.txt" % name)
    with open(path, "w") as f:
        f.write("# %s: exact sampled products, oracle direct sums in __float128 rounded once\n" % name)
        f.write("# written by tests/golden/make_fullsize_quad.py (inputs: workloads.fullsize_case)\n")
        for (i, j), v in zip(st, ds):
            f.write("station %d %d %.17g\n" % (i, j, v))
        for (p, q, rr), v in zip(pq, ts):
            f.write("prism %d %d %d %.17g\n" % (p, q, rr, v))
    print(name, "%.0f s" % (time.time() - t0), path, flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["magnetic_288", "gravity_1024"]:
        write(n)
