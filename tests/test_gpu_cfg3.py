"""The mixed-precision workload end to end on the GPU: FD on the half-filled
Hubbard ring, 64 pairs nearest 0 in [-1, 1], N_s = 256 in bundles of 32,
degree 800, window tracked by the N_t-th Ritz value, FP64 and mixed
precision (FP32 filter; FP64 orthogonalization, Rayleigh-Ritz and residuals).

- L = 12 (D = 853,776): both precisions against the oracle's FD on the same
  start block (tests/golden/hubbard12_fd_oracle.txt, written by the oracle
  alone), eigenvalues within 1e-10 ||H||.
- L = 14 (D = 11,778,624, the dimension of the paper's Hubbard14, Sec. 4.1):
  both precisions converge; every pair agrees between them within
  1e-10 ||H||; residuals recomputed from scratch with the oracle's FP64 SpMMV
  are <= 1e-9 ||H||; the exact level E = 0 (the S_z = 0 member of the fully
  polarised multiplet) is among them; and Lehmann bounds computed from the
  returned vectors prove that the interval spanned by the returned values
  holds at least 64 eigenvalues (completeness of the set, Sec. 2).
"""
import os

import numpy as np
import pytest

import oracle as O
from fd_inputs import start_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hubbard12_fd_oracle.txt")
# one line per FD iteration appended here while the solves run, so that a
# long test shows its progress
_OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
os.makedirs(_OUT, exist_ok=True)
os.environ["FD_TRACE_FILE"] = os.path.join(_OUT, "fd_trace_hubbard_tests.jsonl")
NT, NS, NB, DEG = 64, 256, 32, 800


def golden12():
    with open(GOLDEN) as f:
        return np.array([float(x) for x in f if not x.startswith("#")])


@pytest.mark.parametrize("precision", [0, 1])
def test_hubbard12_matches_oracle_fd(precision):
    want = golden12()
    assert want.size == NT
    m = fd.build_matrix("hubbard", L=12, n_up=6, n_dn=6, t=1.0, U=8.0)
    r = fd.solve(m, -1.0, 1.0, NT, NS, NB, DEG, max_iter=30, tol=1e-9, precision=precision,
                 V0=start_block(m.D, NS, 0), want_vectors=False, adapt=1)
    print("L=12 precision %d: %s" % (precision, r.stats), flush=True)
    assert r.status == fd.FD_OK, r.stats
    normH = r.stats["norm_H"]
    assert np.abs(r.evals - want).max() <= 1e-10 * normH
    assert r.resid.max() <= 1e-9 * normH
    if precision == 1:
        assert r.stats["iters_fp32"] >= 1


@pytest.fixture(scope="module")
def hub14():
    m = fd.build_matrix("hubbard", L=14, n_up=7, n_dn=7, t=1.0, U=8.0)
    runs = {}
    for precision in (0, 1):
        r = fd.solve(m, -1.0, 1.0, NT, NS, NB, DEG, max_iter=20, tol=1e-9, precision=precision, seed=0,
                     want_vectors=True, adapt=1)
        print("L=14 precision %d: %s" % (precision, r.stats), flush=True)
        runs[precision] = r
    yield m, runs
    del runs


def test_hubbard14_both_precisions_converge_and_agree(hub14):
    m, runs = hub14
    r64, rmx = runs[0], runs[1]
    assert r64.status == fd.FD_OK, r64.stats
    assert rmx.status == fd.FD_OK, rmx.stats
    assert rmx.stats["iters_fp32"] >= 1
    normH = r64.stats["norm_H"]
    # per pair: mixed against FP64
    assert np.abs(rmx.evals - r64.evals).max() <= 1e-10 * normH
    # the exact level E = 0 is found
    assert np.abs(r64.evals).min() <= 1e-10 * normH
    assert np.abs(rmx.evals).min() <= 1e-10 * normH


def test_hubbard14_fresh_fp64_residuals(hub14):
    m, runs = hub14
    A = O.hubbard(14, 7, 7, 1.0, 8.0)
    for precision, r in runs.items():
        normH = r.stats["norm_H"]
        X = r.evecs.cpu().numpy()
        fresh = np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0)
        assert fresh.max() <= 1e-9 * normH, (precision, fresh.max() / normH)
        assert np.abs(X.T @ X - np.eye(NT)).max() <= 1e-10
        del X


def test_hubbard14_lehmann_completeness(hub14):
    """Lehmann bounds from the 64 returned vectors, at a shift between 0 and
    the nearest positive returned value, prove at least 64 eigenvalues in
    [-R, R] with R = the largest |lambda| returned (plus the residual slack):
    no eigenvalue nearer 0 can be missing from the set."""
    m, runs = hub14
    r = runs[0]
    normH = r.stats["norm_H"]
    X = r.evecs
    W = torch.empty_like(X)
    fd.spmmv(m, X, W)
    pos = r.evals[r.evals > 1e-8 * normH]
    rho = 0.5 * pos.min()
    lo, up = fd.lehmann(X, W, rho)
    R = np.abs(r.evals).max() + 1e-8 * normH
    n_cert = int(np.sum(lo >= -R)) + int(np.sum(up <= R))
    assert n_cert >= NT, (n_cert, lo[:5], up[:5])
    assert np.all(np.abs(r.evals) <= R)
