"""Write the oracle's eigenvalues for the full-size workloads.

Calls only the seeded generator (jjgen) and the CPU oracle (oracle/).  The
generator is bit-reproducible across hosts, so the stored values belong to the
exact inputs the GPU tests rebuild.  Usage:
    python tests/golden/make_golden.py 2 double      # workload 2, double oracle
    python tests/golden/make_golden.py 3 long        # workload 3, long double oracle
    python tests/golden/make_golden.py 4@1024 long   # workload 4's law downsized to n = 1024
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
    spec = sys.argv[1]
    k, n = (int(spec.split("@")[0]), int(spec.split("@")[1])) if "@" in spec else (int(spec), None)
    prec = sys.argv[2] if len(sys.argv) > 2 else "double"
    G, J, lam = jjgen.config(k, n=n)
    tag = "config%d" % k if n is None else "config%d_n%d" % (k, n)
    t = time.time()
    r = oracle.solve(G, J, precision=prec, vectors=False)
    dt = time.time() - t
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "%s_lambda_%s.txt" % (tag, prec))
    with open(out, "w") as f:
        f.write("# oracle eigenvalues (descending) of workload %d%s, %s working precision\n"
                % (k, "" if n is None else " downsized to n = %d" % n, prec))
        f.write("# written by tests/golden/make_golden.py from jjgen.config(%d%s) and oracle.solve\n"
                % (k, "" if n is None else ", n=%d" % n))
        f.write("# status %d sweeps %d rotations %d seconds %.1f\n" % (r["status"], r["sweeps"], r["rotations"], dt))
        for v in r["lam"]:
            f.write(("%.21Le\n" % v) if False else (np.format_float_scientific(v, precision=20) + "\n"))
    print(out, r["status"], r["sweeps"], dt)


if __name__ == "__main__":
    main()
