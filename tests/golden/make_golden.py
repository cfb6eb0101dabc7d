"""Write the oracle's eigenvalues for the full-size workloads.

Calls only the seeded generator (jjgen) and the CPU oracle (oracle/).  The
generator is bit-reproducible across hosts, so the stored values belong to the
exact inputs the GPU tests rebuild.  Usage:
    python tests/golden/make_golden.py 2 double     # workload 2, double oracle
    python tests/golden/make_golden.py 3 long       # workload 3, long double oracle
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import jjgen  # noqa: E402
import oracle  # noqa: E402


def main():
    k = int(sys.argv[1])
    prec = sys.argv[2] if len(sys.argv) > 2 else "double"
    G, J, lam = jjgen.config(k)
    t = time.time()
    r = oracle.solve(G, J, precision=prec, vectors=False)
    dt = time.time() - t
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config%d_lambda_%s.txt" % (k, prec))
    with open(out, "w") as f:
        f.write("# oracle eigenvalues (descending) of workload %d, %s working precision\n" % (k, prec))
        f.write("# written by tests/golden/make_golden.py from jjgen.config(%d) and oracle.solve\n" % k)
        f.write("# status %d sweeps %d rotations %d seconds %.1f\n" % (r["status"], r["sweeps"], r["rotations"], dt))
        for v in r["lam"]:
            f.write(("%.21Le\n" % v) if False else (np.format_float_scientific(v, precision=20) + "\n"))
    print(out, r["status"], r["sweeps"], dt)


if __name__ == "__main__":
    main()
