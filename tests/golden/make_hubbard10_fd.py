"""Write hubbard10_fd_oracle.txt: the oracle's FD result (CPU, FP64) for the
Hubbard ring L=10, 5 up + 5 down, t=1, U=8: the 16 eigenpairs nearest 0 in
[-1, 1], N_s = 64 (start block N(0,1), seed 0), degree 300, tol 1e-9 relative,
target window tracked during the iteration.  Calls only oracle/.
Run from the repository root: python tests/golden/make_hubbard10_fd.py"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from fd_inputs import start_block  # noqa: E402

A = O.hubbard(10, 5, 5, 1.0, 8.0)
r = O.fd_solve(A, start_block(A.D, 64, 0), -1.0, 1.0, 16, 300, 1e-9, max_iter=60, adapt=True)
assert r.converged
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "hubbard10_fd_oracle.txt"), "w") as f:
    f.write("# oracle FD (tests/golden/make_hubbard10_fd.py): Hubbard L=10 5+5 U=8, 16 pairs nearest 0 in [-1,1]\n")
    f.write("# norm_H %.17g  iterations %d  max residual %.3e\n" % (r.norm_H, r.iters, r.resid.max()))
    for v in r.evals:
        f.write("%.17g\n" % v)
