"""Writes the oracle's per-probe values of the first probes of every
orthogonal tr(D^-1) term (Sec. 3) on the 16^4 two-level workload:
Wilson-clover, c_sw 1, roughness 0.6, m0 0.01, gauge seed 13; 2^4 aggregates,
N_tv 12, test-vector seed 1103; probe seed 103; every solve to a true FP64
relative residual of 1e-12.

Only the oracle runs here (numpy FP64, plain GMRES(50)); the GPU test reads
the file.  It takes about half an hour on one core.

  python tests/golden/make_c3_samples.py [nprobe]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from lattice_inputs import gauge_field  # noqa: E402
from oracle.dirac import WilsonClover  # noqa: E402
from oracle.multigrid import Hierarchy  # noqa: E402
from oracle.solve import gmres  # noqa: E402
from oracle.philox import z4_vector, stream_id, KIND_O, KIND_F, KIND_COARSEST  # noqa: E402

OUT = os.path.join(HERE, "c3_orthogonal_first_probes.txt")


def main():
    nprobe = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    t0 = time.time()
    dims, eps, gseed, m0, csw = (16, 16, 16, 16), 0.6, 13, 0.01, 1.0
    U = gauge_field(dims, eps, gseed)
    D = WilsonClover(U, m0, csw)
    h = Hierarchy(D, [(2, 2, 2, 2)], [12], seed=1103)
    print("hierarchy %.0f s" % (time.time() - t0), flush=True)
    seed = 103

    def solve(l, b):
        return gmres(h.ops[l].matvec, b, tol=1e-12, restart=50)

    tr = h.transfers[0]
    rows = []
    for k in range(nprobe):
        x = z4_vector(h.ops[0].n, seed, stream_id(0, KIND_O), k)
        y = tr.project_out(x)
        X = np.vdot(y, solve(0, y))
        rows.append(("O0", k, X, abs(X)))
        x = z4_vector(h.ops[1].n, seed, stream_id(0, KIND_F), k)
        px = tr.prolong(x)
        a, b = np.vdot(px, solve(0, px)), np.vdot(x, solve(1, x))
        rows.append(("F0", k, a - b, abs(a) + abs(b)))
        x = z4_vector(h.ops[1].n, seed, stream_id(1, KIND_COARSEST), k)
        X = np.vdot(x, solve(1, x))
        rows.append(("coarsest", k, X, abs(X)))
        print("probe %d done %.0f s" % (k, time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle per-probe values X = a - b (and |a| + |b|) of the orthogonal tr(D^-1) terms on\n")
        f.write("# 16^4 Wilson-clover, c_sw 1, roughness 0.6, m0 0.01, gauge seed 13; 2^4 aggregates,\n")
        f.write("# N_tv 12, test-vector seed 1103; probe seed 103; solves to 1e-12 (oracle GMRES(50)).\n")
        f.write("# Written by tests/golden/make_c3_samples.py (oracle only).\n")
        f.write("# term probe re im scale\n")
        for name, k, X, sc in rows:
            f.write("%s %d %.17e %.17e %.17e\n" % (name, k, X.real, X.imag, sc))
    print("wrote", OUT, "%.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
