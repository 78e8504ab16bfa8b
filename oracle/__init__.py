"""Plain FP64 CPU oracle for the filter-diagonalization (FD) hot path.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP library: the sparse parts are plain C loops (fd_oracle.c, loaded with
ctypes), the dense parts are numpy/LAPACK calls in the order the method states.

What it follows (Alvermann, Hager, Fehske, "Orthogonal layers of parallelism in
large-scale eigenvalue computations"):

* Sec. 2, Alg. 1 caption and prose -- the FD iteration: an inclusion interval
  [lam_l, lam_r] for the Chebyshev scaling, a random start block, then
  orthogonalize -> one more SpMV for the Ritz values -> convergence test on the
  N_t best Ritz pairs (rho = ||A v - lam v||_2) -> polynomial filter -> repeat.
* Sec. 2, Alg. 2 caption -- the filter p[A] V with p(x) = sum_k mu_k T_k(x),
  degree n >= 2, n SpMVs, workspaces W1 and W2.
* Sec. 2 -- SVQB orthogonalization from the Gram matrix V^t V (Stathopoulos and
  Wu 2002), used here in place of the paper's TSQR; the two give the same span.
* Sec. 3.1, Eq. SpMVprocess / Eq. traffic -- block SpMV on row-major blocks.

* Sec. 2 -- "a few steps of Lanczos" give the spectral bounds: k steps
  from a seeded start vector, Ritz values of the k x k tridiagonal.

Readings where the paper is silent:
the window function is the indicator of the target interval with Jackson
damping; the inclusion interval for the scaling is Gershgorin's (the
Lanczos interval, widened by the Ritz residuals and 1 % of its width, is the
alternative); ||H|| in the tolerance is the largest |Ritz value| of 40
Lanczos steps, a lower bound of ||H||_2 (so rho <= tol ||H|| is never looser
than the target); the N_t "best" Ritz pairs are those nearest tau inside the
target window.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None


def lib():
    """The compiled oracle; FD_ORACLE_FAST=1 in the environment (read once)
    loads the -O3 x86-64-v3 copy of the same source, which only the
    benchmark's CPU baseline uses."""
    global _lib
    if _lib is None:
        path = _build.build(force=False, fast=os.environ.get("FD_ORACLE_FAST") == "1")
        L = C.CDLL(path)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.orc_num_threads.restype = C.c_int
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.POINTER(C.c_uint64)]
        L.orc_uniform_fill.argtypes = [C.c_uint64, C.c_int64, f64p]
        L.orc_binom.restype = C.c_int64
        L.orc_binom.argtypes = [C.c_int, C.c_int]
        L.orc_hubbard_size.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_hubbard_csr.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                      C.c_double, i64p, u32p, f64p]
        L.orc_anderson_csr.argtypes = [C.c_int, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                       i64p, u32p, f64p]
        L.orc_sell_size.restype = C.c_int64
        L.orc_sell_size.argtypes = [C.c_int64, i64p, C.c_int, C.c_int, i32p, i64p, i32p]
        L.orc_sell_fill.argtypes = [C.c_int64, i64p, u32p, f64p, C.c_int, i32p, i64p,
                                    i32p, u32p, f64p]
        L.orc_spmmv.argtypes = [C.c_int64, i64p, u32p, f64p, C.c_int, C.c_void_p,
                                C.c_int64, C.c_void_p, C.c_int64]
        L.orc_gershgorin.argtypes = [C.c_int64, i64p, u32p, f64p,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_cheb_filter.restype = C.c_int
        L.orc_cheb_filter.argtypes = [C.c_int64, i64p, u32p, f64p, C.c_int, C.c_void_p,
                                      C.c_int64, f64p, C.c_int, C.c_double, C.c_double,
                                      f64p, f64p, f64p, f64p]
        L.orc_jackson.restype = C.c_double
        L.orc_jackson.argtypes = [C.c_int, C.c_int]
        L.orc_cheb_coeffs.restype = C.c_int
        L.orc_cheb_coeffs.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, f64p]
        L.orc_triad.argtypes = [C.c_int64, f64p, f64p, f64p, C.c_double]
        _lib = L
    return _lib


# --------------------------------------------------------------------------- #
# sparse matrices
# --------------------------------------------------------------------------- #
@dataclass
class CSR:
    """Canonical CSR: columns ascending per row, diagonal always stored."""
    D: int
    rowptr: np.ndarray  # int64[D+1]
    col: np.ndarray     # uint32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.D, self.D))
        rows = np.repeat(np.arange(self.D), np.diff(self.rowptr))
        A[rows, self.col.astype(np.int64)] = self.val
        return A


def stream_triad(a: np.ndarray, b: np.ndarray, c: np.ndarray, s: float) -> None:
    """c = a + s b with the oracle's OpenMP threads (the paper's STREAM
    triad, Sec. 3.2, for the host's memory bandwidth b_m)."""
    lib().orc_triad(a.size, a, b, c, s)


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_num_threads())


def splitmix64_first(seed: int, count: int) -> list[int]:
    """The first `count` raw SplitMix64 outputs for `seed`."""
    st = C.c_uint64(seed)
    return [int(lib().orc_splitmix64(C.byref(st))) for _ in range(count)]


def uniforms(seed: int, n: int) -> np.ndarray:
    out = np.empty(n)
    lib().orc_uniform_fill(seed, n, out)
    return out


def binom(n: int, k: int) -> int:
    return int(lib().orc_binom(n, k))


def hubbard(L: int, n_up: int, n_dn: int, t: float = 1.0, U: float = 0.0,
            periodic: bool = True) -> CSR:
    """1D Hubbard ring (or open chain) in the up-major Fock basis."""
    D = C.c_int64()
    nnz = C.c_int64()
    if lib().orc_hubbard_size(L, n_up, n_dn, int(periodic), t, C.byref(D), C.byref(nnz)):
        raise ValueError("invalid Hubbard parameters")
    rowptr = np.empty(D.value + 1, np.int64)
    col = np.empty(nnz.value, np.uint32)
    val = np.empty(nnz.value, np.float64)
    lib().orc_hubbard_csr(L, n_up, n_dn, int(periodic), t, U, rowptr, col, val)
    assert rowptr[-1] == nnz.value
    return CSR(D.value, rowptr, col, val)


def anderson(L: int, t: float = 1.0, W: float = 0.0, seed: int = 1, skip: int = 0) -> CSR:
    """3D Anderson lattice, L^3 sites, periodic, disorder W (u - 1/2), the
    u drawn in row order after the first `skip` draws of SplitMix64(seed)."""
    D = L ** 3
    rowptr = np.empty(D + 1, np.int64)
    col = np.empty(7 * D, np.uint32)
    val = np.empty(7 * D, np.float64)
    if lib().orc_anderson_csr(L, t, W, seed, skip, rowptr, col, val):
        raise ValueError("invalid Anderson parameters")
    return CSR(D, rowptr, col, val)


def diagonal(d: np.ndarray) -> CSR:
    d = np.ascontiguousarray(d, dtype=np.float64)
    D = d.size
    return CSR(D, np.arange(D + 1, dtype=np.int64), np.arange(D, dtype=np.uint32), d.copy())


@dataclass
class SELL:
    D: int
    C: int
    sigma: int
    perm: np.ndarray       # int32[D], perm[new] = old
    chunk_ptr: np.ndarray  # int64[nchunks+1]
    chunk_len: np.ndarray  # int32[nchunks]
    col: np.ndarray        # uint32[total]
    val: np.ndarray        # float64[total]


def sell(A: CSR, C_: int, sigma: int) -> SELL:
    nchunks = (A.D + C_ - 1) // C_
    perm = np.empty(A.D, np.int32)
    cptr = np.empty(nchunks + 1, np.int64)
    clen = np.empty(nchunks, np.int32)
    total = lib().orc_sell_size(A.D, A.rowptr, C_, sigma, perm, cptr, clen)
    if total < 0:
        raise ValueError("invalid SELL parameters")
    col = np.empty(total, np.uint32)
    val = np.empty(total, np.float64)
    lib().orc_sell_fill(A.D, A.rowptr, A.col, A.val, C_, perm, cptr, clen, col, val)
    return SELL(A.D, C_, sigma, perm, cptr, clen, col, val)


def spmmv(A: CSR, X: np.ndarray) -> np.ndarray:
    """Y = A X for a row-major (C-contiguous) D x nb block, FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        return spmmv(A, X[:, None])[:, 0]
    assert X.shape[0] == A.D
    Y = np.empty_like(X)
    nb = X.shape[1]
    lib().orc_spmmv(A.D, A.rowptr, A.col, A.val, nb, X.ctypes.data, nb, Y.ctypes.data, nb)
    return Y


def spmmv_rows(A: CSR, X: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(A X)[rows] row by row from the definition y_i = sum_k A_ik x_k, in CSR
    order (for checking sampled rows of a product too large for the oracle)."""
    out = np.empty((rows.size, X.shape[1]))
    for t, i in enumerate(rows):
        a, b = A.rowptr[i], A.rowptr[i + 1]
        acc = np.zeros(X.shape[1])
        for k in range(a, b):
            acc += A.val[k] * X[A.col[k]]
        out[t] = acc
    return out


def cheb_filter_rows(A: CSR, V: np.ndarray, mu: np.ndarray, alpha: float, beta: float,
                     rows: np.ndarray) -> np.ndarray:
    """(p[alpha A + beta] V)[rows]: the same recurrence as cheb_filter, carried
    only on the rows each step needs (row set of step k = rows of step k+1
    plus their neighbours), so that sampled rows of a large filter can be
    computed exactly as the definition states."""
    n = mu.size - 1
    sets = [np.unique(rows)]
    for _ in range(n):
        r = sets[-1]
        nbr = np.concatenate([A.col[A.rowptr[i]:A.rowptr[i + 1]].astype(np.int64) for i in r])
        sets.append(np.union1d(r, nbr))
    sets = sets[::-1]  # sets[k]: rows where T_k is needed (T_k on sets[k])

    def take(T, have, want):
        return T[np.searchsorted(have, want)]

    def apply_B(T, have, want):  # (alpha A + beta) T on rows `want`
        out = np.empty((want.size, T.shape[1]))
        for t, i in enumerate(want):
            acc = np.zeros(T.shape[1])
            for k in range(A.rowptr[i], A.rowptr[i + 1]):
                acc += A.val[k] * T[np.searchsorted(have, A.col[k])]
            out[t] = alpha * acc + beta * T[np.searchsorted(have, i)]
        return out

    final = sets[-1]
    T0 = V[sets[0]].astype(np.float64)
    T1 = apply_B(T0, sets[0], sets[1])
    S = mu[0] * take(T0, sets[0], final) + mu[1] * take(T1, sets[1], final)
    prev, prevset, cur, curset = T0, sets[0], T1, sets[1]
    for k in range(2, n + 1):
        nxt = 2.0 * apply_B(cur, curset, sets[k]) - take(prev, prevset, sets[k])
        S += mu[k] * take(nxt, sets[k], final)
        prev, prevset, cur, curset = cur, curset, nxt, sets[k]
    return S[np.searchsorted(final, rows)]


def kpm_moments(A: CSR, R: np.ndarray, nmom: int, alpha: float, beta: float) -> np.ndarray:
    """mu_k = (1/(nR D)) sum_r <r|T_k(alpha A + beta)|r>, k < nmom, by the plain
    recurrence T_{k+1} r = 2 B T_k r - T_{k-1} r (no doubling)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    D, nr = R.shape
    mu = np.empty(nmom)
    T0 = R.copy()
    T1 = alpha * spmmv(A, T0) + beta * T0
    mu[0] = np.sum(R * T0) / (nr * D)
    if nmom > 1:
        mu[1] = np.sum(R * T1) / (nr * D)
    for k in range(2, nmom):
        T2 = 2.0 * (alpha * spmmv(A, T1) + beta * T1) - T0
        mu[k] = np.sum(R * T2) / (nr * D)
        T0, T1 = T1, T2
    return mu


def gershgorin(A: CSR) -> tuple[float, float]:
    lo = C.c_double()
    hi = C.c_double()
    lib().orc_gershgorin(A.D, A.rowptr, A.col, A.val, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


LANCZOS_STEPS = 40
LANCZOS_SEED = 1


def lanczos(A: CSR, k: int = LANCZOS_STEPS, seed: int = LANCZOS_SEED):
    """k steps of Lanczos (Sec. 2: spectral bounds from a few Lanczos steps)
    with full reorthogonalization (classical Gram-Schmidt against all
    previous vectors, applied twice), from the start vector u_i = 2 U_i - 1,
    U_i the i-th uniform of SplitMix64(seed) (i from 0).  Stops early when
    the new vector's norm falls to 1e-12 of the largest |alpha| (an invariant
    subspace).  Returns (theta ascending, resid = beta_k |s_kj|, steps)."""
    D = A.D
    k = max(1, min(k, D))
    q = 2.0 * uniforms(seed, D) - 1.0
    q /= np.linalg.norm(q)
    Q = np.zeros((D, k))
    alpha = np.zeros(k)
    beta = np.zeros(k)
    steps = k
    for j in range(k):
        Q[:, j] = q
        w = spmmv(A, q[:, None])[:, 0]
        for _ in range(2):
            c = Q[:, :j + 1].T @ w
            w = w - Q[:, :j + 1] @ c
            alpha[j] += c[j]
        beta[j] = np.linalg.norm(w)
        if beta[j] <= 1e-12 * np.abs(alpha[:j + 1]).max():
            steps = j + 1
            break
        q = w / beta[j]
    T = np.diag(alpha[:steps]) + np.diag(beta[:steps - 1], 1) + np.diag(beta[:steps - 1], -1)
    theta, S = np.linalg.eigh(T)
    resid = beta[steps - 1] * np.abs(S[steps - 1, :])
    return theta, resid, steps


def lanczos_norm(A: CSR) -> float:
    """||H|| of the tolerance: the largest |Ritz value| of lanczos(A)."""
    theta, _, _ = lanczos(A)
    return float(max(abs(theta[0]), abs(theta[-1])))


def lanczos_interval(A: CSR, k: int, seed: int = LANCZOS_SEED) -> tuple[float, float]:
    """Inclusion interval from k Lanczos steps: the extreme Ritz values moved
    out by their residual bounds and by 1 % of the resulting width."""
    theta, resid, _ = lanczos(A, k, seed)
    lo, hi = theta[0] - resid[0], theta[-1] + resid[-1]
    w = 0.01 * (hi - lo)
    return lo - w, hi + w


def scaling(lam_l: float, lam_r: float) -> tuple[float, float]:
    """alpha, beta that map [lam_l, lam_r] onto [-1, 1] (Alg. 2 caption)."""
    return 2.0 / (lam_r - lam_l), -(lam_r + lam_l) / (lam_r - lam_l)


def jackson(n: int, k: int) -> float:
    return float(lib().orc_jackson(n, k))


def cheb_coeffs(kind: int, a: float, b: float, n: int) -> np.ndarray:
    """kind 0: Jackson-damped indicator of [a,b]; kind 1: damped delta at a."""
    mu = np.empty(n + 1)
    if lib().orc_cheb_coeffs(kind, a, b, n, mu):
        raise ValueError("invalid coefficient request")
    return mu


def cheb_filter(A: CSR, V: np.ndarray, mu: np.ndarray, alpha: float, beta: float) -> np.ndarray:
    """Return p[A] V for p(x) = sum_k mu_k T_k(alpha x + beta); V is D x nb."""
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    if V.ndim == 1:
        return cheb_filter(A, V[:, None], mu, alpha, beta)[:, 0]
    D, nb = V.shape
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n = mu.size - 1
    T0, T1, T2, AX = (np.empty((D, nb)) for _ in range(4))
    got = lib().orc_cheb_filter(D, A.rowptr, A.col, A.val, nb, V.ctypes.data, nb, mu, n,
                                alpha, beta, T0, T1, T2, AX)
    if got != n:
        raise ValueError("filter degree must be >= 2")
    return V


# --------------------------------------------------------------------------- #
# dense steps (numpy / LAPACK as library primitives)
# --------------------------------------------------------------------------- #
def svqb(V: np.ndarray, clip: float = 1e-14) -> tuple[np.ndarray, int]:
    """One SVQB pass (Stathopoulos & Wu 2002): G = V^t V, Dg = diag(G)^-1/2,
    Dg G Dg = U L U^t, V <- V Dg U L^-1/2 with L clipped at clip * max(L).
    Returns the new block and the number of unclipped eigenvalues."""
    G = V.T @ V
    G = 0.5 * (G + G.T)
    d = np.sqrt(np.diag(G))
    d[d == 0] = 1.0
    Dg = 1.0 / d
    Gs = Dg[:, None] * G * Dg[None, :]
    lam, U = np.linalg.eigh(Gs)
    floor = clip * max(lam.max(), 0.0)
    rank = int(np.sum(lam > floor))
    lam = np.maximum(lam, floor) if floor > 0 else np.where(lam > 0, lam, 1.0)
    Q = (Dg[:, None] * U) / np.sqrt(lam)[None, :]
    return V @ Q, rank


def svqb2(V: np.ndarray, clip: float = 1e-14) -> tuple[np.ndarray, int]:
    V1, rank = svqb(V, clip)
    V2, _ = svqb(V1, clip)
    return V2, rank


def rayleigh_ritz(A: CSR, V: np.ndarray):
    """W = A V (the one extra SpMV), H = V^t W, H = Y diag(theta) Y^t, rotate
    V and W to the Ritz basis, rho_j = ||W_j - theta_j V_j||_2."""
    W = spmmv(A, V)
    H = V.T @ W
    H = 0.5 * (H + H.T)
    theta, Y = np.linalg.eigh(H)
    Vr = V @ Y
    Wr = W @ Y
    rho = np.linalg.norm(Wr - Vr * theta[None, :], axis=0)
    return theta, Vr, Wr, rho


def select_targets(theta: np.ndarray, tau_lo: float, tau_hi: float, n_target: int) -> np.ndarray:
    """Indices of the n_target Ritz values nearest tau = (tau_lo+tau_hi)/2 that lie
    in [tau_lo, tau_hi] (all Ritz values nearest tau when tau_lo == tau_hi);
    ties go to the lower value."""
    tau = 0.5 * (tau_lo + tau_hi)
    idx = np.arange(theta.size)
    if tau_hi > tau_lo:
        idx = idx[(theta >= tau_lo) & (theta <= tau_hi)]
    order = sorted(idx.tolist(), key=lambda j: (abs(theta[j] - tau), theta[j]))
    return np.array(order[:n_target], dtype=np.int64)


@dataclass
class FDResult:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray
    converged: bool
    iters: int
    spmmv_cols: int          # SpMV count per column (filter degree sum + RR)
    norm_H: float
    history: list = field(default_factory=list)


def lehmann(A: CSR, V: np.ndarray, rho: float):
    """Lehmann's inclusion intervals (Lehmann 1963) for the shift rho from the
    subspace spanned by the columns of V; the paper determines its target and
    search intervals from them (Sec. 2).

    With M0 = V^t V, M1 = V^t A V, M2 = (AV)^t (AV), the eigenvalues mu of
    the definite pencil (M1 - rho M0) x = mu (M2 - 2 rho M1 + rho^2 M0) x
    give: for the i-th most negative mu, [rho + 1/mu, rho) holds at least i
    eigenvalues of A; for the i-th largest positive mu, (rho, rho + 1/mu]
    holds at least i.  Returns (lower, upper, mu) with lower and upper in
    that order (nearest rho first)."""
    import scipy.linalg
    AV = spmmv(A, V)
    M0 = V.T @ V
    M1 = V.T @ AV
    M1 = 0.5 * (M1 + M1.T)
    M2 = AV.T @ AV
    mu = scipy.linalg.eigh(M1 - rho * M0, M2 - 2.0 * rho * M1 + rho * rho * M0, eigvals_only=True)
    lower = rho + 1.0 / mu[mu < 0]
    upper = rho + 1.0 / mu[mu > 0][::-1]
    return lower, upper, mu


def lehmann_radius(lower: np.ndarray, upper: np.ndarray, rho: float, k: int) -> float:
    """Smallest r such that the Lehmann intervals certify k eigenvalues in
    [rho - r, rho + r] (left and right counts add: the intervals are
    disjoint); inf if fewer than k are certified."""
    d = np.sort(np.concatenate([rho - lower, upper - rho]))
    return float(d[k - 1]) if d.size >= k else float("inf")


def fd_solve(A: CSR, V0: np.ndarray, tau_lo: float, tau_hi: float, n_target: int,
             degree: int, tol: float = 1e-9, max_iter: int = 50, adapt: int = 0, interval: int = 0) -> FDResult:
    """Plain FD (Alg. 1 reading) with a fixed degree and fixed target window.

    [lam_l, lam_r] = Gershgorin interval; alpha, beta from it; ||H|| =
    lanczos_norm(A).  Loop: V <- SVQB2(V); Rayleigh-Ritz; if the n_target
    pairs nearest tau in the window all have rho <= tol * ||H||, stop; else
    V <- p[A] V with the Jackson-damped indicator of the scaled window (a
    damped delta at tau when tau_lo == tau_hi).  With adapt, the filter's
    window is shrunk each iteration to tau +- the distance of the n_target-th
    nearest Ritz value in the window (the target interval is tracked during
    the iteration, Sec. 2); with adapt == 2 to tau +- the Lehmann radius,
    which provably holds n_target eigenvalues.  interval = k > 0 scales with
    the k-step Lanczos interval (inside Gershgorin's) instead.
    """
    lam_l, lam_r = gershgorin(A)
    if interval > 0:  # k-step Lanczos interval, inside Gershgorin's
        a, b = lanczos_interval(A, interval)
        lam_l, lam_r = max(lam_l, a), min(lam_r, b)
    alpha, beta = scaling(lam_l, lam_r)
    norm_H = lanczos_norm(A)
    if tau_hi > tau_lo:
        mu = cheb_coeffs(0, alpha * tau_lo + beta, alpha * tau_hi + beta, degree)
    else:
        mu = cheb_coeffs(1, alpha * tau_lo + beta, 0.0, degree)
    V = np.array(V0, dtype=np.float64, order="C", copy=True)
    spmv = 0
    hist = []
    it = 0
    while True:
        V, _ = svqb2(V)
        theta, V, W, rho = rayleigh_ritz(A, V)
        spmv += 1
        sel = select_targets(theta, tau_lo, tau_hi, n_target)
        ok = sel.size == n_target and bool(np.all(rho[sel] <= tol * norm_H))
        hist.append(float(rho[sel].max()) if sel.size else float("inf"))
        if ok or it >= max_iter:
            order = sel[np.argsort(theta[sel], kind="stable")]
            return FDResult(theta[order], V[:, order], rho[order], ok, it, spmv, norm_H, hist)
        tau = 0.5 * (tau_lo + tau_hi)
        r = None
        if adapt == 1 and tau_hi > tau_lo and sel.size == n_target:
            r = abs(theta[sel[-1]] - tau)
        if adapt == 2 and tau_hi > tau_lo:
            lo_l, up_l, _ = lehmann(A, V, tau)
            r = lehmann_radius(lo_l, up_l, tau, n_target)
            r = r if np.isfinite(r) else None
        if r is not None:
            lo_w, hi_w = max(tau_lo, tau - r), min(tau_hi, tau + r)
            a = min(1.0, max(-1.0, alpha * lo_w + beta))
            b = max(a, min(1.0, alpha * hi_w + beta))
            mu = cheb_coeffs(0, a, b, degree)
        V = cheb_filter(A, V, mu, alpha, beta)
        spmv += degree
        it += 1
