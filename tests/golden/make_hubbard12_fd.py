"""Write hubbard12_fd_oracle.txt: the oracle's FD result (CPU, FP64) for the
Hubbard ring L=12, 6 up + 6 down, t=1, U=8 (D = 853,776): the 64 eigenpairs
nearest 0 in [-1, 1], N_s = 256 (start block N(0,1), seed 0), degree 800,
tol 1e-9 relative, target window tracked during the iteration (the Hubbard
L=14 workload one size down, where the oracle still finishes on a CPU).
Calls only oracle/.  Run from the repository root (about an hour on 8 cores):
python tests/golden/make_hubbard12_fd.py"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from fd_inputs import start_block  # noqa: E402

t0 = time.time()
A = O.hubbard(12, 6, 6, 1.0, 8.0)
r = O.fd_solve(A, start_block(A.D, 256, 0), -1.0, 1.0, 64, 800, 1e-9, max_iter=30, adapt=True)
assert r.converged
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "hubbard12_fd_oracle.txt"), "w") as f:
    f.write("# oracle FD (tests/golden/make_hubbard12_fd.py): Hubbard L=12 6+6 U=8, 64 pairs nearest 0 in [-1,1],"
            " N_s=256, degree 800\n")
    f.write("# norm_H %.17g  iterations %d  max residual %.3e  (%.0f s)\n"
            % (r.norm_H, r.iters, r.resid.max(), time.time() - t0))
    for v in r.evals:
        f.write("%.17g\n" % v)
