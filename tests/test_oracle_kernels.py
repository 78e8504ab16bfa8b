"""Pins for the oracle's SpMMV, Chebyshev filter, coefficients, SVQB, Rayleigh-Ritz
and FD loop (CPU only)."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy import integrate

import oracle as O
from fd_inputs import int_block, start_block


# ----------------------------------------------------------------- SpMMV ----
@pytest.mark.parametrize("nb", [1, 3, 8, 16])
def test_spmmv_vs_dense_matmul(nb):
    A = O.hubbard(7, 3, 3, 1.0, 2.5)
    X = start_block(A.D, nb, 5)
    np.testing.assert_allclose(O.spmmv(A, X), A.dense() @ X, rtol=0, atol=1e-12)


def test_spmmv_integer_exact():
    A = O.anderson(6, 1.0, 0.0)
    X = int_block(A.D, 8, 2)
    Y = O.spmmv(A, X)
    Yref = (A.dense().astype(np.int64) @ X.astype(np.int64)).astype(np.float64)
    assert np.array_equal(Y, Yref)


# ---------------------------------------------------------- coefficients ----
def test_jackson_normalisation_and_first_factor():
    for n in (2, 10, 100, 800):
        assert abs(O.jackson(n, 0) - 1.0) < 1e-15
        N = n + 1
        assert abs(O.jackson(n, 1) - math.cos(math.pi / (N + 1))) < 1e-15


def test_jackson_kernel_positive_and_width():
    """The Jackson-damped delta is a positive kernel of unit mass whose variance
    at x = 0 approaches (pi / N)^2 (Weisse et al. RMP 2006)."""
    n = 60
    N = n + 1
    x = np.cos(np.linspace(0, np.pi, 2001))
    for y in (-0.7, 0.0, 0.31, 0.95):
        mu = O.cheb_coeffs(1, y, 0.0, n)
        p = npcheb.chebval(x, mu)
        assert p.min() > -1e-12 * p.max()
    mu0 = O.cheb_coeffs(1, 0.0, 0.0, 400)
    # <x^2> under the weight 1/(pi sqrt(1-x^2)): x^2 = (T0 + T2)/2 and
    # <T_k> = mu_k (1 + delta_k0)/2
    var = 0.5 * (mu0[0] + 0.5 * mu0[2])
    assert abs(var / (math.pi / 401) ** 2 - 1) < 0.02


@pytest.mark.parametrize("a,b", [(-0.3, 0.2), (-1.0, -0.9), (0.05, 0.06)])
def test_indicator_coefficients_by_quadrature(a, b):
    n = 40
    mu = O.cheb_coeffs(0, a, b, n)
    for k in range(n + 1):
        ck = integrate.quad(lambda th: math.cos(k * th), math.acos(b), math.acos(a),
                            epsabs=1e-14)[0] * (1 if k == 0 else 2) / math.pi
        assert abs(mu[k] - O.jackson(n, k) * ck) < 1e-13


def test_window_polynomial_bounds_and_limit():
    n = 400
    mu = O.cheb_coeffs(0, -0.2, 0.3, n)
    x = np.linspace(-1, 1, 4001)
    p = npcheb.chebval(x, mu)
    assert p.min() > -1e-12 and p.max() < 1 + 1e-12
    # Jackson tails decay algebraically: ~1e-5 at a quarter-width inside,
    # ~1e-7 half the window away from an edge at n = 400
    assert abs(npcheb.chebval(0.05, mu) - 1) < 1e-4
    assert abs(npcheb.chebval(0.8, mu)) < 1e-5


# ---------------------------------------------------------------- filter ----
def test_filter_chebyshev_identity():
    """mu = e_n on diag(cos theta) gives T_n(cos theta) = cos(n theta)."""
    theta = np.linspace(0.01, 3.1, 300)
    A = O.diagonal(np.cos(theta))
    V = start_block(A.D, 4, 1)
    for n in (2, 3, 17, 100):
        mu = np.zeros(n + 1)
        mu[n] = 1.0
        out = O.cheb_filter(A, V, mu, 1.0, 0.0)
        np.testing.assert_allclose(out, np.cos(n * theta)[:, None] * V, atol=1e-11)


def test_filter_diagonal_clenshaw():
    lam = np.linspace(-3.0, 5.0, 257)
    A = O.diagonal(lam)
    alpha, beta = O.scaling(-3.0, 5.0)
    mu = O.cheb_coeffs(0, -0.1, 0.2, 50)
    V = start_block(A.D, 3, 2)
    out = O.cheb_filter(A, V, mu, alpha, beta)
    np.testing.assert_allclose(out, npcheb.chebval(alpha * lam + beta, mu)[:, None] * V,
                               atol=1e-12)


def test_filter_general_matrix_via_eigendecomposition():
    A = O.hubbard(6, 3, 3, 1.0, 4.0)
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    mu = O.cheb_coeffs(0, alpha * -1 + beta, alpha * 1 + beta, 60)
    lam, Q = np.linalg.eigh(A.dense())
    V = start_block(A.D, 5, 3)
    want = Q @ (npcheb.chebval(alpha * lam + beta, mu)[:, None] * (Q.T @ V))
    got = O.cheb_filter(A, V, mu, alpha, beta)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want) + 1e-13


def test_filter_rejects_degree_below_two():
    A = O.diagonal(np.ones(4))
    with pytest.raises(ValueError):
        O.cheb_filter(A, np.ones((4, 1)), np.ones(2), 1.0, 0.0)


# ------------------------------------------------------------ SVQB / RR ----
def test_svqb2_orthonormal_span_and_rank():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((3000, 40)) @ np.diag(np.logspace(0, -6, 40))
    Q, rank = O.svqb2(V)
    assert rank == 40
    assert np.abs(Q.T @ Q - np.eye(40)).max() < 1e-13
    assert np.linalg.norm(V - Q @ (Q.T @ V)) <= 1e-12 * np.linalg.norm(V)
    W = np.concatenate([V[:, :10], V[:, :10]], axis=1)
    _, r2 = O.svqb(W)
    assert r2 == 10


def test_rayleigh_ritz_exact_on_eigenvectors():
    lam = np.linspace(-2, 2, 50)
    A = O.diagonal(lam)
    idx = [3, 17, 30, 44]
    V = np.eye(50)[:, idx]
    theta, Vr, Wr, rho = O.rayleigh_ritz(A, V)
    np.testing.assert_allclose(theta, lam[idx], atol=1e-15)
    assert rho.max() < 1e-15


def test_rayleigh_ritz_residuals_recomputed():
    A = O.anderson(5, 1.0, 8.0)
    V, _ = O.svqb2(start_block(A.D, 12, 4))
    theta, Vr, Wr, rho = O.rayleigh_ritz(A, V)
    fresh = np.linalg.norm(A.dense() @ Vr - Vr * theta, axis=0)
    np.testing.assert_allclose(rho, fresh, atol=1e-13)


# ---------------------------------------------------------------- FD loop ----
def test_select_targets_window_and_ties():
    th = np.array([-0.3, -0.1, 0.1, 0.2, 0.6, -0.6])
    assert list(O.select_targets(th, -0.5, 0.5, 3)) == [1, 2, 3]
    assert list(O.select_targets(th, -0.5, 0.5, 9)) == [1, 2, 3, 0]
    assert list(O.select_targets(th, 0.0, 0.0, 2)) == [1, 2]


def test_fd_fig2_diagonal_search_interval():
    """Fig. 2: 1000 equidistant eigenvalues, N_t = 10, N_s = 20, target
    [-0.01, 0.01].  A filter whose Jackson broadening fits the search interval
    [-0.02, 0.02] converges; one sized for [-0.04, 0.04] (more than N_s
    eigenvalues inside) does not within 20 iterations."""
    lam = -1 + 2 * np.arange(1000) / 999
    A = O.diagonal(lam)
    V0 = start_block(1000, 20, 0)
    for delta, ok in ((0.01, True), (0.03, False)):
        n = math.ceil(math.pi * 2 / (2 * delta)) - 2
        r = O.fd_solve(A, V0, -0.01, 0.01, 10, n, 1e-9, max_iter=20)
        assert r.converged == ok
        if ok:
            want = lam[(lam >= -0.01) & (lam <= 0.01)]
            np.testing.assert_allclose(r.evals, want, atol=1e-12)


@pytest.mark.slow
def test_fd_hubbard8_vs_dense():
    """Hubbard L=8 (4 up, 4 down, U = 4): 16 eigenpairs nearest 0 in [-0.5, 0.5],
    degree 100, N_s = 128, checked against dense diagonalisation."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = np.linalg.eigvalsh(A.dense())
    r = O.fd_solve(A, start_block(A.D, 128, 0), -0.5, 0.5, 16, 100, 1e-9, max_iter=80)
    assert r.converged
    want = np.sort(ev[np.argsort(np.abs(ev), kind="stable")[:16]])
    assert np.abs(r.evals - want).max() <= 1e-10 * r.norm_H
    assert r.resid.max() <= 1e-9 * r.norm_H
    fresh = np.linalg.norm(O.spmmv(A, r.evecs) - r.evecs * r.evals, axis=0)
    assert fresh.max() <= 1e-9 * r.norm_H


def test_row_sampled_forms_match_full_oracle():
    A = O.anderson(7, 1.0, 16.5, 2)
    X = start_block(A.D, 5, 1)
    rows = np.array([0, 3, 100, 342, 17, 17 * 7 + 2])
    np.testing.assert_array_equal(O.spmmv_rows(A, X, rows), O.spmmv(A, X)[rows])
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    mu = O.cheb_coeffs(1, 0.1, 0.0, 4)
    full = O.cheb_filter(A, X, mu, alpha, beta)
    np.testing.assert_allclose(O.cheb_filter_rows(A, X, mu, alpha, beta, rows), full[rows], rtol=0, atol=1e-13)


def test_kpm_moments_exact_trace():
    """With the full unit basis scaled by sqrt(D) (so that the average of r r^t
    is I, as for N(0,1) vectors) the stochastic trace is exact:
    mu_k = (1/D) sum_i T_k(alpha lambda_i + beta)."""
    A = O.hubbard(6, 2, 3, 1.0, 2.0)
    lam = np.linalg.eigvalsh(A.dense())
    alpha, beta = O.scaling(*O.gershgorin(A))
    x = alpha * lam + beta
    mu = O.kpm_moments(A, np.sqrt(A.D) * np.eye(A.D), 12, alpha, beta)
    want = [np.mean(np.cos(k * np.arccos(np.clip(x, -1, 1)))) for k in range(12)]
    np.testing.assert_allclose(mu, want, atol=1e-13)
    assert abs(mu[0] - 1.0) < 1e-15


def test_mlp_oracle_gradient_by_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(3)
    p = mlp.init(1, out_scale=1.0)
    X = rng.uniform(-1, 1, (6, 66))
    Y = rng.standard_normal((6, 2))
    w = np.array([1.0, 0.5])
    loss, g = mlp.loss_and_grad(p, X, Y, w)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (mlp.loss_and_grad(p + e, X, Y, w)[0] - mlp.loss_and_grad(p - e, X, Y, w)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    assert p.size == 41858


# ------------------------------------------------------------ Lehmann bounds --
def test_lehmann_exact_on_eigenvectors():
    """With V spanning exact eigenvectors, every bound is one of their
    eigenvalues: the pencil is diagonal with mu = 1/(lambda - rho)."""
    A = O.hubbard(6, 3, 3, 1.0, 4.0)
    lam, X = np.linalg.eigh(A.dense())
    idx = np.array([10, 40, 120, 121, 200, 300])
    rho = 0.5 * (lam[121] + lam[122])  # in the gap above the degenerate pair 120, 121
    assert lam[122] - lam[121] > 1e-3
    lower, upper, _ = O.lehmann(A, X[:, idx], rho)
    below = np.sort(lam[idx][lam[idx] < rho])[::-1]
    above = np.sort(lam[idx][lam[idx] > rho])
    np.testing.assert_allclose(lower, below, atol=1e-10 * 24)
    np.testing.assert_allclose(upper, above, atol=1e-10 * 24)


def test_lehmann_single_vector_is_the_temple_kato_bound():
    """One vector v (|v| = 1), Rayleigh quotient theta < rho, residual r:
    the bound is theta - r^2 / (rho - theta) (worked out by hand from the
    pencil: mu = (theta - rho) / ((theta - rho)^2 + r^2))."""
    A = O.anderson(6, 1.0, 8.0, 4)
    v = start_block(A.D, 1, 5)
    v /= np.linalg.norm(v)
    Av = O.spmmv(A, v)
    theta = float(v[:, 0] @ Av[:, 0])
    r2 = float(np.sum((Av - theta * v) ** 2))
    rho = theta + 0.7
    lower, upper, _ = O.lehmann(A, v, rho)
    assert upper.size == 0 and lower.size == 1
    assert abs(lower[0] - (theta - r2 / (rho - theta))) <= 1e-12 * (1 + abs(lower[0]))


@pytest.mark.parametrize("name,k,rho", [("and6", 24, 0.0), ("and6", 40, 1.3), ("hub6", 30, 2.01), ("hub6", 12, -4.4)])
def test_lehmann_bounds_hold_against_dense_spectrum(name, k, rho):
    """The theorem: [lower[i], rho) and (rho, upper[i]] each hold at least
    i+1 eigenvalues; the radius certifies k_t eigenvalues in rho +- r.  V is
    a random block after a few filter steps, so bounds are far from exact."""
    A = O.anderson(6, 1.0, 8.0, 4) if name == "and6" else O.hubbard(6, 3, 3, 1.0, 4.0)
    lam = np.linalg.eigvalsh(A.dense())
    assert np.min(np.abs(lam - rho)) > 1e-6
    alpha, beta = O.scaling(*O.gershgorin(A))
    V = O.cheb_filter(A, start_block(A.D, k, 8), O.cheb_coeffs(1, alpha * rho + beta, 0.0, 12), alpha, beta)
    V, _ = O.svqb2(V)
    lower, upper, mu = O.lehmann(A, V, rho)
    assert lower.size + upper.size == k
    for i, b in enumerate(lower):
        assert np.sum((lam >= b) & (lam < rho)) >= i + 1
    for i, b in enumerate(upper):
        assert np.sum((lam > rho) & (lam <= b)) >= i + 1
    for kt in (1, 4, 8):
        r = O.lehmann_radius(lower, upper, rho, kt)
        assert np.sum(np.abs(lam - rho) <= r) >= kt
        # and it is no smaller than the exact kt-th distance
        assert r >= np.sort(np.abs(lam - rho))[kt - 1] - 1e-12


def test_fd_lehmann_window_hubbard8_vs_dense():
    """FD with the Lehmann-controlled window converges to the dense answer."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    r = O.fd_solve(A, start_block(A.D, 128, 0), -0.5, 0.5, 16, 100, 1e-9, max_iter=80, adapt=2)
    assert r.converged
    ev = np.linalg.eigvalsh(A.dense())
    inside = ev[(ev >= -0.5) & (ev <= 0.5)]
    want = np.sort(inside[np.argsort(np.abs(inside), kind="stable")[:16]])
    assert np.abs(r.evals - want).max() <= 1e-10 * r.norm_H


# --------------------------------------------------------------- Lanczos ----
def test_lanczos_exact_when_krylov_space_is_whole():
    """D <= k: the Krylov space is the whole space, so the Ritz values are the
    eigenvalues (distinct diagonal) and the residual bounds vanish."""
    d = np.linspace(-3.0, 5.0, 23) ** 3 / 10.0
    A = O.diagonal(d)
    th, rs, steps = O.lanczos(A, 40, 1)
    assert steps == 23
    np.testing.assert_allclose(th, np.sort(d), rtol=0, atol=1e-12)
    assert rs.max() <= 1e-10


def test_lanczos_stops_at_an_invariant_subspace():
    """Three distinct levels: the start vector lies in a 3-dimensional
    invariant subspace, so Lanczos stops after 3 steps with the 3 levels."""
    d = np.repeat([-1.0, 0.5, 2.0], 7)
    th, rs, steps = O.lanczos(O.diagonal(d), 40, 1)
    assert steps == 3
    np.testing.assert_allclose(th, [-1.0, 0.5, 2.0], rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", ["hub8", "and8"])
def test_lanczos_ritz_values_against_dense_spectrum(name):
    """Cauchy interlacing: every Ritz value lies inside [lam_min, lam_max];
    each Ritz value has an eigenvalue within its residual bound; the extreme
    ones converge first (40 steps: within 1e-6 relative)."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0) if name == "hub8" else O.anderson(8, 1.0, 8.0, 4)
    lam = np.linalg.eigvalsh(A.dense())
    th, rs, steps = O.lanczos(A, 40, 1)
    assert steps == 40
    assert th.min() >= lam[0] - 1e-12 and th.max() <= lam[-1] + 1e-12
    dist = np.abs(th[:, None] - lam[None, :]).min(axis=1)
    assert np.all(dist <= rs + 1e-12)
    normH = max(abs(lam[0]), abs(lam[-1]))
    assert abs(th[0] - lam[0]) <= 1e-6 * normH and abs(th[-1] - lam[-1]) <= 1e-6 * normH
    est = O.lanczos_norm(A)
    assert est <= normH * (1 + 1e-14) and est >= normH * (1 - 1e-6)
    lo, hi = O.lanczos_interval(A, 40)
    assert lo <= lam[0] and hi >= lam[-1]


def test_lanczos_norm_is_tighter_than_gershgorin():
    """Hubbard L=8, U=4: the Gershgorin bound is 32 against ||H||_2 = 20.6;
    the Lanczos estimate sits just below ||H||_2 (a lower bound; 40 steps
    bring it within about 1e-8 here)."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    lam = np.linalg.eigvalsh(A.dense())
    normH = max(abs(lam[0]), abs(lam[-1]))
    assert max(abs(x) for x in O.gershgorin(A)) == 32.0
    est = O.lanczos_norm(A)
    assert est <= normH and normH - est <= 1e-6 * normH
