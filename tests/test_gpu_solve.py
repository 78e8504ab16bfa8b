"""End-to-end FD (fd_solve) on the GPU against the oracle and dense spectra."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from fd_inputs import start_block
from lattice_walk import anderson_tiled, tile_walk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402

_DENSE = {}


def dense_spectrum(key, A):
    if key not in _DENSE:
        _DENSE[key] = np.linalg.eigvalsh(A.dense())
    return _DENSE[key]


def nearest(ev, tau_lo, tau_hi, k):
    tau = 0.5 * (tau_lo + tau_hi)
    inside = ev[(ev >= tau_lo) & (ev <= tau_hi)]
    order = sorted(range(inside.size), key=lambda j: (abs(inside[j] - tau), inside[j]))
    return np.sort(inside[order[:k]])


def check_pairs(A, r, want, normH):
    assert np.abs(r.evals - want).max() <= 1e-10 * normH
    assert r.resid.max() <= 1e-9 * normH
    X = r.evecs.cpu().numpy()
    fresh = np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0)
    assert fresh.max() <= 1e-9 * normH
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("fmt,C_,sigma", [("csr", 1, 1), ("sell", 32, 512)])
def test_hubbard8_vs_dense(precision, fmt, C_, sigma):
    """Hubbard L=8 (4+4, U=4): 16 pairs nearest 0 in [-0.5, 0.5], degree 100,
    N_s = 128 in bundles of 16, start block N(0,1) seed 0."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = dense_spectrum("hub8", A)
    m = fd.build_matrix("hubbard", fmt=fmt, C_=C_, sigma=sigma, L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, precision=precision,
                 V0=start_block(A.D, 128, 0))
    assert r.status == fd.FD_OK, r.stats
    check_pairs(A, r, nearest(ev, -0.5, 0.5, 16), r.stats["norm_H"])
    if precision == 1:
        assert r.stats["iters_fp32"] >= 1


def test_hubbard8_matches_oracle_fd():
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    V0 = start_block(A.D, 128, 0)
    ro = O.fd_solve(A, V0, -0.5, 0.5, 16, 100, 1e-9, max_iter=80)
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, V0=V0)
    assert ro.converged and r.status == fd.FD_OK
    assert np.abs(r.evals - ro.evals).max() <= 1e-10 * ro.norm_H


def test_hubbard8_U0_closed_form():
    L, N = 8, 4
    eps = -2.0 * np.cos(2 * np.pi * np.arange(L) / L)
    sums = [sum(eps[list(s)]) for s in itertools.combinations(range(L), N)]
    spec = np.sort(np.add.outer(sums, sums).ravel())
    m = fd.build_matrix("hubbard", L=L, n_up=N, n_dn=N, t=1.0, U=0.0)
    A = O.hubbard(L, N, N, 1.0, 0.0)
    # the bottom of the spectrum: a 4-fold and a 16-fold level (20 in the window)
    r = fd.solve(m, -10.5, -8.0, 8, 64, 16, 120, max_iter=80, tol=1e-9, V0=start_block(A.D, 64, 1))
    assert r.status == fd.FD_OK, r.stats
    check_pairs(A, r, nearest(spec, -10.5, -8.0, 8), r.stats["norm_H"])


def test_hubbard8_particle_hole_mirror():
    """Half filling: lambda -> U L / 2 - lambda maps the spectrum onto itself."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    r1 = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, V0=start_block(A.D, 128, 0))
    r2 = fd.solve(m, 15.5, 16.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, V0=start_block(A.D, 128, 3))
    assert r1.status == fd.FD_OK and r2.status == fd.FD_OK
    np.testing.assert_allclose(np.sort(16.0 - r2.evals), r1.evals, atol=1e-10 * r1.stats["norm_H"])


def test_fig2_diagonal_search_interval():
    lam = -1 + 2 * np.arange(1000) / 999
    m = fd.build_matrix("diagonal", diag=lam)
    V0 = start_block(1000, 20, 0)
    for delta, ok in ((0.01, True), (0.03, False)):
        n = math.ceil(math.pi * 2 / (2 * delta)) - 2
        r = fd.solve(m, -0.01, 0.01, 10, 20, 4, n, max_iter=20, tol=1e-9, V0=V0)
        assert (r.status == fd.FD_OK) == ok
        if ok:
            np.testing.assert_allclose(r.evals, lam[(lam >= -0.01) & (lam <= 0.01)], atol=1e-12)
        else:
            assert r.status == fd.FD_ERR_NOT_CONVERGED and r.stats["iters"] <= 20


def test_library_start_block_and_determinism():
    A = O.hubbard(6, 3, 3, 1.0, 4.0)
    ev = dense_spectrum("hub6", A)
    m = fd.build_matrix("hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0)
    r1 = fd.solve(m, -0.5, 0.5, 4, 32, 8, 60, max_iter=60, seed=42)
    r2 = fd.solve(m, -0.5, 0.5, 4, 32, 8, 60, max_iter=60, seed=42)
    assert r1.status == fd.FD_OK
    check_pairs(A, r1, nearest(ev, -0.5, 0.5, 4), r1.stats["norm_H"])
    assert np.array_equal(r1.evals, r2.evals) and np.array_equal(r1.resid, r2.resid)
    assert torch.equal(r1.evecs, r2.evecs)


def test_anderson_nearest_tau_delta_filter():
    """tau_lo == tau_hi selects the pairs nearest tau with the damped delta."""
    A = O.anderson(12, 1.0, 16.5, 1)
    ev = dense_spectrum("and12", A)
    m = fd.build_matrix("anderson", L=12, t=1.0, W=16.5, seed=1)
    r = fd.solve(m, 0.0, 0.0, 8, 64, 16, 400, max_iter=100, tol=1e-9, V0=start_block(A.D, 64, 2))
    assert r.status == fd.FD_OK, r.stats
    want = np.sort(ev[np.argsort(np.abs(ev), kind="stable")[:8]])
    check_pairs(A, r, want, r.stats["norm_H"])


def test_anderson_tiled_numbering_same_pairs():
    """The tiled site numbering is P A P^T: the same eigenvalues nearest 0
    as the dense natural spectrum, and eigenvectors that are the tiled
    matrix's own (checked with a fresh SpMMV of the permuted oracle matrix)
    and, mapped back through the walk, the natural matrix's."""
    A = O.anderson(12, 1.0, 16.5, 1)
    ev = dense_spectrum("and12", A)
    B = anderson_tiled(12, 1.0, 16.5, 1, 5, 4)
    m = fd.build_matrix("anderson", L=12, t=1.0, W=16.5, seed=1, tiles=(5, 4))
    r = fd.solve(m, 0.0, 0.0, 8, 64, 16, 400, max_iter=100, tol=1e-9, V0=start_block(A.D, 64, 2))
    assert r.status == fd.FD_OK, r.stats
    want = np.sort(ev[np.argsort(np.abs(ev), kind="stable")[:8]])
    check_pairs(B, r, want, r.stats["norm_H"])
    X = np.empty_like(r.evecs.cpu().numpy())
    X[tile_walk(12, 5, 4)] = r.evecs.cpu().numpy()  # row r of the walk is site walk[r]
    assert np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0).max() <= 1e-9 * r.stats["norm_H"]


def test_solve_errors_and_not_converged():
    m = fd.build_matrix("hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0)
    with pytest.raises(fd.FDError) as e:
        fd.solve(m, -100.0, 0.5, 4, 32, 8, 60)
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError):
        fd.solve(m, -0.5, 0.5, 4, 36, 8, 60)  # N_s not a multiple of nb
    with pytest.raises(fd.FDError):
        fd.solve(m, -0.5, 0.5, 40, 32, 8, 60)  # N_t > N_s
    r = fd.solve(m, -0.5, 0.5, 4, 32, 8, 60, max_iter=1, seed=1)
    assert r.status == fd.FD_ERR_NOT_CONVERGED
    assert r.stats["iters"] == 1 and np.all(np.isfinite(r.evals))
    assert r.stats["spmmv_count"] == 2 * (32 // 8) + 60 * (32 // 8)


def test_hubbard8_adaptive_window_vs_dense():
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = dense_spectrum("hub8", A)
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    for prec in (0, 1):
        r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, precision=prec,
                     V0=start_block(A.D, 128, 0), adapt=1)
        assert r.status == fd.FD_OK, r.stats
        check_pairs(A, r, nearest(ev, -0.5, 0.5, 16), r.stats["norm_H"])


def test_hubbard10_adaptive_vs_oracle_fd():
    """Hubbard L=10 (D = 63,504): beyond dense size; against the oracle's FD
    (tests/golden/hubbard10_fd_oracle.txt, written by make_hubbard10_fd.py),
    with fresh FP64 residual certificates."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "hubbard10_fd_oracle.txt")
    want = np.array([float(x) for x in open(path) if x.strip() and not x.startswith("#")])
    A = O.hubbard(10, 5, 5, 1.0, 8.0)
    m = fd.build_matrix("hubbard", L=10, n_up=5, n_dn=5, t=1.0, U=8.0)
    for prec in (0, 1):
        r = fd.solve(m, -1.0, 1.0, 16, 64, 16, 300, max_iter=60, tol=1e-9, precision=prec,
                     V0=start_block(A.D, 64, 0), adapt=1)
        assert r.status == fd.FD_OK, r.stats
        normH = r.stats["norm_H"]
        assert np.abs(r.evals - want).max() <= 1e-10 * normH
        X = r.evecs.cpu().numpy()
        fresh = np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0)
        assert fresh.max() <= 1e-9 * normH
        assert np.min(np.abs(r.evals)) < 1e-10 * normH  # the exact E = 0 level
