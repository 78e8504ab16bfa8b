"""GPU parity of libfd's kernels against the CPU oracle (through the C ABI).

Tolerances: FP64 results within 1e-12 relative (Frobenius) of the oracle;
bit-exact where every partial sum is an exact integer; FP32 results within a
bound derived from the FP32 unit roundoff times the accumulation length.
"""
import numpy as np
import pytest

import oracle as O
from fd_inputs import int_block, start_block
from lattice_walk import anderson_tiled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


MATS = {
    "hub8": (dict(model="hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0), lambda: O.hubbard(8, 4, 4, 1.0, 4.0)),
    "hub7": (dict(model="hubbard", L=7, n_up=3, n_dn=2, t=1.0, U=2.5), lambda: O.hubbard(7, 3, 2, 1.0, 2.5)),
    "and13": (dict(model="anderson", L=13, t=1.0, W=16.5, seed=1), lambda: O.anderson(13, 1.0, 16.5, 1)),
    # sites numbered along (x, y) tiles of 5 x 4 (ragged at the lattice edge)
    "and12t": (dict(model="anderson", L=12, t=1.0, W=16.5, seed=1, tiles=(5, 4)),
               lambda: anderson_tiled(12, 1.0, 16.5, 1, 5, 4)),
}
FMTS = [("csr", 1, 1), ("sell", 32, 256), ("sell", 64, 1), ("sell", 8, 1 << 20)]


def build(name, fmt, C_, sigma):
    kw, ora = MATS[name]
    return fd.build_matrix(fmt=fmt, C_=C_, sigma=sigma, **kw), ora()


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("fmt,C_,sigma", FMTS)
@pytest.mark.parametrize("nb", [1, 2, 4, 8, 16, 32, 64])
def test_spmmv_fp64_parity(name, fmt, C_, sigma, nb):
    m, A = build(name, fmt, C_, sigma)
    X = start_block(A.D, nb, 11)
    Y = torch.empty((A.D, nb), dtype=torch.float64, device="cuda")
    fd.spmmv(m, dev(X), Y)
    torch.cuda.synchronize()
    assert relerr(Y.cpu().numpy(), O.spmmv(A, X)) <= 1e-12


@pytest.mark.parametrize("name", ["hub8", "and13", "and12t"])
@pytest.mark.parametrize("fmt,C_,sigma", FMTS[:2])
@pytest.mark.parametrize("nb", [1, 4, 8, 64])
def test_spmmv_integer_bit_exact(name, fmt, C_, sigma, nb):
    kw, _ = MATS[name]
    if name == "and13":
        kw = dict(kw, W=0.0)  # integer values
        A = O.anderson(13, 1.0, 0.0, 1)
    elif name == "and12t":
        kw = dict(kw, W=0.0)
        A = anderson_tiled(12, 1.0, 0.0, 1, 5, 4)
    else:
        A = MATS[name][1]()
    m = fd.build_matrix(fmt=fmt, C_=C_, sigma=sigma, **kw)
    for dt, bound in ((torch.float64, 1 << 10), (torch.float32, 1 << 8)):
        X = int_block(A.D, nb, 3, bound)
        Y = torch.empty((A.D, nb), dtype=dt, device="cuda")
        fd.spmmv(m, dev(X, dt), Y)
        torch.cuda.synchronize()
        assert np.array_equal(Y.cpu().double().numpy(), O.spmmv(A, X))


@pytest.mark.parametrize("nb", [1, 8, 64])
def test_spmmv_fp32_error_bound(nb):
    m, A = build("hub8", "csr", 1, 1)
    X = start_block(A.D, nb, 5)
    X32 = X.astype(np.float32)
    Y = torch.empty((A.D, nb), dtype=torch.float32, device="cuda")
    fd.spmmv(m, dev(X32), Y)
    torch.cuda.synchronize()
    # |fl(sum) - sum| <= len * u * sum |a x| with u = 2^-24 and len <= 17
    Aabs = O.CSR(A.D, A.rowptr, A.col, np.abs(A.val))
    bound = 17 * 2.0 ** -24 * O.spmmv(Aabs, np.abs(X32.astype(np.float64)))
    ref = O.spmmv(A, X32.astype(np.float64))
    assert np.all(np.abs(Y.cpu().double().numpy() - ref) <= bound + 1e-30)


def test_spmmv_ld_and_errors():
    m, A = build("hub7", "csr", 1, 1)
    X = start_block(A.D, 16, 1)
    Xd = torch.zeros((A.D, 24), dtype=torch.float64, device="cuda")
    Xd[:, 4:12] = dev(X[:, :8])
    Y = torch.full((A.D, 10), 7.0, dtype=torch.float64, device="cuda")
    fd.spmmv(m, Xd[:, 4:12], Y[:, :8])
    torch.cuda.synchronize()
    assert relerr(Y[:, :8].cpu().numpy(), O.spmmv(A, X[:, :8])) <= 1e-12
    assert torch.all(Y[:, 8:] == 7.0)
    with pytest.raises(fd.FDError):
        fd.spmmv(m, Xd[:, :3], torch.empty((A.D, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(fd.FDError):  # misaligned (odd element offset, FP64 needs 16 bytes)
        fd.spmmv(m, Xd[:, 1:9], Y[:, :8])


# ------------------------------------------------------------------ filter --
@pytest.mark.parametrize("name", ["hub8", "and13", "and12t"])
@pytest.mark.parametrize("fmt,C_,sigma", FMTS[:2])
@pytest.mark.parametrize("nb,nbund,concurrent", [(1, 2, False), (8, 3, True), (16, 2, False), (64, 1, False)])
def test_filter_fp64_parity(name, fmt, C_, sigma, nb, nbund, concurrent):
    m, A = build(name, fmt, C_, sigma)
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    mu = O.cheb_coeffs(0, alpha * -0.5 + beta, alpha * 0.5 + beta, 37)
    ns = nb * nbund
    V = start_block(A.D, ns, 2)
    ldw = ns if concurrent else nb
    Vd = dev(V)
    W1 = torch.empty((A.D, ldw), dtype=torch.float64, device="cuda")
    W2 = torch.empty_like(W1)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, nb)
    torch.cuda.synchronize()
    assert relerr(Vd.cpu().numpy(), O.cheb_filter(A, V, mu, alpha, beta)) <= 1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 50])
def test_filter_chebyshev_identity(n):
    theta = np.linspace(0.01, 3.1, 999)
    m = fd.build_matrix("diagonal", diag=np.cos(theta))
    V = start_block(999, 8, 4)
    mu = np.zeros(n + 1)
    mu[n] = 1.0
    Vd = dev(V)
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, 1.0, 0.0, W1, W2, 8)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Vd.cpu().numpy(), np.cos(n * theta)[:, None] * V, atol=1e-12)


def test_filter_fp32_error():
    m, A = build("hub8", "csr", 1, 1)
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    mu = O.cheb_coeffs(0, alpha * -0.5 + beta, alpha * 0.5 + beta, 100)
    V = start_block(A.D, 16, 6).astype(np.float32)
    Vd = dev(V)
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, 16)
    torch.cuda.synchronize()
    ref = O.cheb_filter(A, V.astype(np.float64), mu, alpha, beta)
    # an FP32 recurrence of degree n loses about n * 2^-24 relative
    assert relerr(Vd.cpu().double().numpy(), ref) <= 100 * 2.0 ** -24 * 10


# -------------------------------------------------------------- dense FP64 --
@pytest.mark.parametrize("D,m_,n", [(10007, 64, 64), (5001, 17, 33), (4096, 256, 256), (333, 1, 5),
                                    (70000, 128, 100), (2000, 512, 512), (70001, 300, 130), (123457, 512, 512),
                                    (9, 128, 128)])
def test_gram_parity_and_reproducible(D, m_, n):
    X = start_block(D, m_, 1)
    Y = start_block(D, n, 2)
    G = torch.empty((m_, n), dtype=torch.float64, device="cuda")
    fd.gram(dev(X), dev(Y), G)
    g1 = G.cpu().numpy()
    ref = X.T @ Y
    assert np.abs(g1 - ref).max() <= 1e-13 * np.sqrt(D) * max(1.0, np.abs(ref).max()) / 10
    fd.gram(dev(X), dev(Y), G)
    assert np.array_equal(G.cpu().numpy(), g1)


@pytest.mark.parametrize("D,m_,n", [(10007, 64, 64), (5001, 17, 9), (4096, 256, 256), (999, 300, 300),
                                    (3000, 512, 512), (50, 20, 1)])
def test_rotate_parity(D, m_, n):
    X = start_block(D, m_, 3)
    Q = start_block(m_, n, 4)
    Xd = dev(X)
    fd.rotate(Xd, dev(Q))
    out = Xd.cpu().numpy()
    ref = X @ Q
    assert np.abs(out[:, :n] - ref).max() <= 1e-13 * np.sqrt(m_) * np.abs(ref).max()
    assert np.array_equal(out[:, n:], X[:, n:])


@pytest.mark.parametrize("n", [1, 2, 5, 64, 127, 128, 200, 256, 512])
def test_syev_parity(n):
    rng = np.random.default_rng(n)
    S = rng.standard_normal((n, n))
    S = S + S.T
    if n >= 64:  # exact multiplicities, as in Ritz matrices of symmetric models
        lam, Q = np.linalg.eigh(S)
        lam[: n // 4] = 1.5
        S = (Q * lam) @ Q.T
        S = 0.5 * (S + S.T)
    Sd = dev(S)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    U = torch.empty((n, n), dtype=torch.float64, device="cuda")
    fd.syev(Sd, w, U)
    wn, Un = w.cpu().numpy(), U.cpu().numpy()
    ref = np.linalg.eigvalsh(S)
    nrm = np.linalg.norm(S, 2)
    assert np.abs(wn - ref).max() <= 1e-13 * nrm * max(1, np.sqrt(n) / 4)
    assert np.abs(Un.T @ Un - np.eye(n)).max() <= 1e-13 * max(1, n / 64)
    assert np.abs(S @ Un - Un * wn).max() <= 1e-12 * nrm * max(1, n / 64)


@pytest.mark.parametrize("method", [fd.FD_ORTHO_SVQB2, fd.FD_ORTHO_CHOLQR2])
@pytest.mark.parametrize("D,ns", [(5000, 64), (20011, 128), (6000, 129), (3000, 16), (40000, 256), (2000, 1)])
def test_orthog(method, D, ns):
    V = start_block(D, ns, 9) @ np.diag(np.logspace(0, -5, ns))
    Vd = dev(V)
    r = fd.orthog(Vd, method)
    Q = Vd.cpu().numpy()
    assert r == ns
    assert np.abs(Q.T @ Q - np.eye(ns)).max() <= 1e-13
    assert np.linalg.norm(V - Q @ (Q.T @ V)) <= 1e-11 * np.linalg.norm(V)


def test_orthog_rank_deficient_refill():
    D, ns = 4000, 32
    V = start_block(D, ns, 1)
    V[:, 20:] = V[:, :12]  # 12 duplicated columns
    Vd = dev(V)
    r = fd.orthog(Vd, fd.FD_ORTHO_SVQB2, seed=5)
    Q = Vd.cpu().numpy()
    assert r == 20
    assert np.abs(Q.T @ Q - np.eye(ns)).max() <= 1e-13
    # the kept span contains the original columns
    assert np.linalg.norm(V - Q @ (Q.T @ V)) <= 1e-11 * np.linalg.norm(V)


@pytest.mark.parametrize("name,nb,ns", [("hub8", 16, 64), ("and13", 8, 40), ("hub7", 4, 12)])
def test_rayleigh_ritz_parity(name, nb, ns):
    m, A = build(name, "csr", 1, 1)
    V, _ = O.svqb2(start_block(A.D, ns, 8))
    th_o, Vr_o, Wr_o, rho_o = O.rayleigh_ritz(A, V)
    Vd = dev(V)
    Wd = torch.empty_like(Vd)
    th, rho = fd.rayleigh_ritz(m, Vd, Wd, nb)
    normH = max(abs(m.lam_lo), abs(m.lam_hi))
    assert np.abs(th - th_o).max() <= 1e-12 * normH
    assert np.abs(rho - rho_o).max() <= 1e-11 * normH
    Vn = Vd.cpu().numpy()
    fresh = np.linalg.norm(O.spmmv(A, Vn) - Vn * th, axis=0)
    assert np.abs(fresh - rho).max() <= 1e-11 * normH


@pytest.mark.parametrize("n", [1 << 20, (1 << 20) + 6, 2050])
def test_stream_kernels_exact(n):
    a = torch.arange(n, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    fd.stream(0, a, c)
    assert torch.equal(c, a)
    fd.stream(1, a, c, b, 0.5)
    assert torch.equal(c, a + 1.5)


@pytest.mark.parametrize("order,xcd,iters,grid,nt,wide,shfl", [(0, 1, 0, 0, 0, 0, 0), (0, 0, 4, 0, 1, 0, 0),
                                                               (1, 1, 0, 1024, 1, 0, 0), (1, 0, 0, 96, 0, 0, 0),
                                                               (0, 2, 1, 64, 1, 1, 0), (0, 0, 1, 0, 1, 1, 0),
                                                               (0, 2, 1, 1024, 1, 0, 1), (1, 1, 0, 512, 0, 0, 1),
                                                               (0, 2, 1, 2048, 1, 1, 1), (0, 2, 1, 1024, 1, 0, 2),
                                                               (0, 2, 1, 8192, 1, 0, 1), (1, 1, 0, 512, 0, 1, 2),
                                                               (1, 0, 0, 96, 1, 1, 2)])
def test_launch_shapes_give_identical_results(order, xcd, iters, grid, nt, wide, shfl):
    """Every launch shape computes each row the same way: bitwise equal."""
    m, A = build("hub8", "sell", 32, 256)
    X = dev(start_block(A.D, 16, 1))
    Y0 = torch.empty_like(X)
    fd.spmmv(m, X, Y0)
    try:
        fd.spmmv_tune(order, xcd, iters, grid, nt, wide, 0, shfl)
        Y1 = torch.empty_like(X)
        fd.spmmv(m, X, Y1)
        lo, hi = O.gershgorin(A)
        alpha, beta = O.scaling(lo, hi)
        mu = O.cheb_coeffs(0, -0.2, 0.2, 9)
        V = dev(start_block(A.D, 32, 2))
        W1 = torch.empty_like(V)
        W2 = torch.empty_like(V)
        fd.cheb_filter(m, V, mu, alpha, beta, W1, W2, 16)
        torch.cuda.synchronize()
    finally:
        fd.spmmv_tune()
    assert torch.equal(Y0, Y1)
    assert relerr(V.cpu().numpy(), O.cheb_filter(A, start_block(A.D, 32, 2), mu, alpha, beta)) <= 1e-12


def test_autotune_keeps_results():
    m, A = build("and13", "csr", 1, 1)
    X = dev(start_block(A.D, 8, 3))
    Y0 = torch.empty_like(X)
    fd.spmmv(m, X, Y0)
    shape = fd.autotune(m, "f64", 8)
    assert shape[0] in (0, 1) and shape[1] in (0, 1, 2) and shape[4] in (0, 1)
    Y1 = torch.empty_like(X)
    fd.spmmv(m, X, Y1)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)


@pytest.mark.parametrize("name,nb,nmom", [("hub8", 16, 64), ("and13", 8, 32), ("hub7", 1, 10)])
def test_kpm_moments_parity(name, nb, nmom):
    m, A = build(name, "csr", 1, 1)
    alpha, beta = O.scaling(*O.gershgorin(A))
    R = start_block(A.D, nb, 31)
    mu = fd.kpm_moments(m, dev(R), nmom, alpha, beta)
    ref = O.kpm_moments(A, R, nmom, alpha, beta)
    # doubling vs direct recurrence: equal up to rounding
    assert np.abs(mu - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_kpm_window_count_exact_basis():
    A = O.hubbard(6, 3, 3, 1.0, 4.0)
    lam = np.linalg.eigvalsh(A.dense())
    m = fd.build_matrix("hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0)
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = fd.kpm_moments(m, dev(np.sqrt(A.D) * np.eye(A.D)), 400, alpha, beta)  # exact trace
    est = fd.window_count(mu, A.D, alpha * -2.0 + beta, alpha * 2.0 + beta)
    true = np.sum((lam >= -2.0) & (lam <= 2.0))
    assert abs(est - true) <= 0.05 * true + 3


def test_mlp_forward_and_gradient_vs_oracle():
    from oracle import mlp
    rng = np.random.default_rng(7)
    p = mlp.init(2, out_scale=0.5)
    X = rng.uniform(-1, 1, (37, 66))
    Y = rng.standard_normal((37, 2))
    w = np.array([1.0, 0.3])
    P = torch.from_numpy(p.astype(np.float32)).cuda()
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    out = torch.empty((37, 2), dtype=torch.float32, device="cuda")
    fd.mlp_forward(P, Xd, out)
    ref, _, _ = mlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    G = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    fd.mlp_grad(P, Xd, torch.from_numpy(Y.astype(np.float32)).cuda(), torch.from_numpy(w.astype(np.float32)).cuda(),
                G, loss)
    lref, gref = mlp.loss_and_grad(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
                                   Y.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64))
    assert abs(float(loss.item()) - lref) <= 1e-4 * max(1.0, lref)
    gn = G.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gn - gref) <= 1e-3 * np.linalg.norm(gref)


def test_mlp_adam_step_matches_formula():
    n = 41858
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    P, G = torch.from_numpy(p0.copy()).cuda(), torch.from_numpy(g).cuda()
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    fd.mlp_adam(P, G, M, V, 1, 1e-2, 0.1)
    m1 = 0.1 * g
    v1 = 0.001 * g * g
    want = p0 - 1e-2 * ((m1 / 0.1) / (np.sqrt(v1 / 0.001) + 1e-8) + 0.1 * p0)
    np.testing.assert_allclose(P.cpu().numpy(), want, rtol=1e-5, atol=1e-6)


def test_pick_degree_rule_hubbard8():
    """The KPM rule's radii bracket the dense N_t-th and N_s-th nearest
    eigenvalue distances, and fd_solve with degree 0 converges."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = np.sort(np.abs(np.linalg.eigvalsh(A.dense())))
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    deg, r, feat = fd.pick_degree(m, -0.5, 0.5, 16, 128, seed=1)
    assert 20 <= deg <= 20000 and feat.shape == (66,)
    assert 0.5 * ev[15] <= r <= 2.0 * ev[15] + 0.1
    res = fd.solve(m, -0.5, 0.5, 16, 128, 16, 0, max_iter=80, tol=1e-9, V0=start_block(A.D, 128, 0), adapt=1)
    assert res.status == fd.FD_OK
    assert 0.7 * deg <= res.stats["degree"] <= 1.4 * deg  # its own KPM draw


@pytest.mark.parametrize("L,tx,ty", [(13, 16, 16), (13, 4, 3), (20, 8, 8), (7, 1, 7)])
def test_pencil_order_bitwise_equal_to_csr(L, tx, ty):
    """The pencil walk changes only the order of the rows, not a row's
    arithmetic: SpMMV and filter (every step form) equal CSR bit for bit,
    and the filter matches the oracle."""
    kw = dict(L=L, t=1.0, W=16.5, seed=1)
    mc = fd.build_matrix("anderson", **kw)
    mp = fd.build_matrix("anderson", fmt="pencil", C_=tx, sigma=ty, **kw)
    A = O.anderson(L, 1.0, 16.5, 1)
    for dt in (torch.float64, torch.float32):
        X = dev(start_block(A.D, 16, 1), dt)
        Yc, Yp = torch.empty_like(X), torch.empty_like(X)
        fd.spmmv(mc, X, Yc)
        fd.spmmv(mp, X, Yp)
        alpha, beta = O.scaling(*O.gershgorin(A))
        for degree in (9, 10):
            mu = O.cheb_coeffs(1, beta, 0.0, degree)
            V0 = dev(start_block(A.D, 32, 2), dt)
            Vc, Vp = V0.clone(), V0.clone()
            W1, W2 = torch.empty_like(V0), torch.empty_like(V0)
            fd.cheb_filter(mc, Vc, mu, alpha, beta, W1, W2, 16)
            fd.cheb_filter(mp, Vp, mu, alpha, beta, W1, W2, 16)
            torch.cuda.synchronize()
            assert torch.equal(Vc, Vp)
            if dt == torch.float64:
                ref = O.cheb_filter(A, V0.cpu().numpy(), mu, alpha, beta)
                assert relerr(Vp.cpu().numpy(), ref) <= 1e-12
        assert torch.equal(Yc, Yp)


def _arrow(D, seed):
    """Arrow matrix: row 0 couples to every row (D entries), every other row
    holds only its diagonal and column 0 -- the most uneven row lengths."""
    rng = np.random.default_rng(seed)
    rowptr = np.zeros(D + 1, np.int64)
    cols, vals = [], []
    for i in range(D):
        c = np.arange(D) if i == 0 else np.array([0, i])
        v = rng.integers(-3, 4, size=c.size).astype(np.float64)
        cols.append(c)
        vals.append(v)
        rowptr[i + 1] = rowptr[i] + c.size
    col = np.concatenate(cols).astype(np.uint32)
    val = np.concatenate(vals)
    # symmetric: A[i][0] = A[0][i]
    for i in range(1, D):
        val[rowptr[i]] = val[i]
    return O.CSR(D, rowptr, col, val)


@pytest.mark.parametrize("fmt,C_,sigma", [("csr", 1, 1), ("sell", 32, 256), ("sell", 8, 1)])
@pytest.mark.parametrize("nb", [1, 8, 64])
def test_ragged_rows_arrow_matrix(fmt, C_, sigma, nb):
    """Row lengths 1003 and 2 in one matrix (one ragged SELL chunk against
    full ones): SpMMV bit-exact on integers, filter within 1e-12."""
    A = _arrow(1003, 4)
    m = fd.build_matrix("csr", fmt=fmt, C_=C_, sigma=sigma, csr=(A.rowptr, A.col, A.val))
    X = int_block(A.D, nb, 6, 1 << 10)
    Y = torch.empty((A.D, nb), dtype=torch.float64, device="cuda")
    fd.spmmv(m, dev(X), Y)
    torch.cuda.synchronize()
    assert np.array_equal(Y.cpu().numpy(), O.spmmv(A, X))
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(0, -0.3, 0.4, 11)
    V = start_block(A.D, nb, 7)
    Vd = dev(V)
    W1, W2 = torch.empty_like(Vd), torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, nb)
    torch.cuda.synchronize()
    assert relerr(Vd.cpu().numpy(), O.cheb_filter(A, V, mu, alpha, beta)) <= 1e-12


@pytest.mark.parametrize("nb", [1, 2, 64])
def test_one_row_matrix(nb):
    """D = 1: the smallest matrix every kernel must take."""
    m = fd.build_matrix("diagonal", diag=np.array([0.75]))
    X = dev(np.full((1, nb), 2.0))
    Y = torch.empty_like(X)
    fd.spmmv(m, X, Y)
    V = dev(np.full((1, nb), 1.0))
    W1, W2 = torch.empty_like(V), torch.empty_like(V)
    mu = O.cheb_coeffs(1, 0.2, 0.0, 6)
    alpha, beta = 0.8, -0.1  # the Gershgorin interval of a 1 x 1 matrix is a point
    fd.cheb_filter(m, V, mu, alpha, beta, W1, W2, nb)
    torch.cuda.synchronize()
    assert torch.all(Y == 1.5)
    want = O.cheb_filter(O.diagonal(np.array([0.75])), np.ones((1, nb)), mu, alpha, beta)
    assert relerr(V.cpu().numpy(), want) <= 1e-14


def test_solve_full_search_space():
    """N_s = D: the search space is the whole space, so one Rayleigh-Ritz
    gives exact pairs (no filter step is needed)."""
    d = np.linspace(-1.0, 1.0, 16)
    m = fd.build_matrix("diagonal", diag=d)
    r = fd.solve(m, -0.3, 0.3, 4, 16, 8, 10, max_iter=5, tol=1e-9, V0=start_block(16, 16, 1))
    assert r.status == fd.FD_OK and r.stats["iters"] == 0
    want = np.sort(d[np.argsort(np.abs(d), kind="stable")[:4]])
    assert np.abs(r.evals - want).max() <= 1e-13


# --------------------------------------------------------------- Lanczos ----
@pytest.mark.parametrize("name,k", [("hub8", 40), ("and8", 40), ("diag", 60), ("hub6", 7)])
def test_lanczos_matches_oracle(name, k):
    """fd_lanczos against the oracle's Lanczos (same seeded start vector,
    full reorthogonalization): same number of steps, Ritz values within
    1e-10 ||H||, residual bounds within 1e-10 ||H|| (absolute)."""
    if name == "hub8":
        A, m = O.hubbard(8, 4, 4, 1.0, 4.0), fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    elif name == "hub6":
        A, m = O.hubbard(6, 3, 3, 1.0, 4.0), fd.build_matrix("hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0)
    elif name == "and8":
        A, m = O.anderson(8, 1.0, 8.0, 4), fd.build_matrix("anderson", L=8, t=1.0, W=8.0, seed=4)
    else:
        d = np.linspace(-2.0, 3.0, 45)
        A, m = O.diagonal(d), fd.build_matrix("diagonal", diag=d)
    th, rs = fd.lanczos(m, k, 1)
    tho, rso, steps = O.lanczos(A, k, 1)
    assert th.size == steps
    normH = max(abs(tho[0]), abs(tho[-1]))
    assert np.abs(th - tho).max() <= 1e-10 * normH
    assert np.abs(rs - rso).max() <= 1e-10 * normH


def test_solve_uses_lanczos_norm_and_interval():
    """fd_solve's ||H|| is the 40-step Lanczos estimate (the oracle's), a
    lower bound of ||H||_2; with interval = 30 the Lanczos interval scales the
    filter and the result still matches dense diagonalization."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    lam = np.linalg.eigvalsh(A.dense())
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    V0 = start_block(A.D, 128, 0)
    inside = lam[(lam >= -0.5) & (lam <= 0.5)]
    want = np.sort(inside[np.argsort(np.abs(inside), kind="stable")[:16]])
    for interval in (0, 30):
        r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, V0=V0, interval=interval)
        assert r.status == fd.FD_OK, r.stats
        normH = r.stats["norm_H"]
        assert abs(normH - O.lanczos_norm(A)) <= 1e-12 * normH
        assert normH <= max(abs(lam[0]), abs(lam[-1]))
        assert np.abs(r.evals - want).max() <= 1e-10 * normH
        assert r.resid.max() <= 1e-9 * normH
        ro = O.fd_solve(A, V0, -0.5, 0.5, 16, 100, 1e-9, max_iter=80, interval=interval)
        assert ro.converged and np.abs(ro.evals - r.evals).max() <= 1e-10 * normH


@pytest.mark.parametrize("lpr", [4, 8, 16])
@pytest.mark.parametrize("name", ["hub8", "and13", "and12t"])
def test_one_vector_lane_shared_rows(lpr, name):
    """nb = 1 on CSR with lpr lanes per row (coalesced entry loads, partial
    sums added across lanes): SpMMV within 1e-12 of the oracle and bit-exact
    on integer data when the matrix is integer (Hubbard); every step form of the filter (first steps, V every
    other step, an odd last step) within 1e-12 in FP64 and at FP32 rounding
    in FP32."""
    m, A = build(name, "csr", 1, 1)
    try:
        fd.spmmv_tune(lpr=lpr)
        X = start_block(A.D, 1, 3)
        Y = torch.empty((A.D, 1), dtype=torch.float64, device="cuda")
        fd.spmmv(m, dev(X), Y)
        assert relerr(Y.cpu().numpy(), O.spmmv(A, X)) <= 1e-12
        if np.array_equal(A.val, np.round(A.val)):  # integer matrix: every order of the sum is exact
            Xi = int_block(A.D, 1, 4)
            fd.spmmv(m, dev(Xi), Y)
            assert np.array_equal(Y.cpu().numpy(), O.spmmv(A, Xi))
        lo, hi = O.gershgorin(A)
        alpha, beta = O.scaling(lo, hi)
        for deg in (2, 3, 10, 11):
            mu = O.cheb_coeffs(0, -0.3, 0.25, deg)
            V0 = start_block(A.D, 4, 5)
            ref = O.cheb_filter(A, V0, mu, alpha, beta)
            for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
                V = dev(V0, dt)
                W1, W2 = torch.empty_like(V), torch.empty_like(V)
                fd.cheb_filter(m, V, mu, alpha, beta, W1, W2, 1)
                assert relerr(V.cpu().double().numpy(), ref) <= tol, (deg, dt)
    finally:
        fd.spmmv_tune()


@pytest.mark.parametrize("nb,shfl", [(8, 1), (16, 2), (64, 1), (64, 2)])
def test_uniform_rows_variant_matches_the_wave_exchange(nb, shfl):
    """Anderson rows all hold 7 entries, so the step kernel skips the
    exchange of row lengths across the wave (a compile-time variant).  The
    same matrix with one explicit zero added to row 0 has rows of two
    lengths and takes the exchange.  The added entry contributes fma(0, x,
    acc) = acc, so every output is bitwise equal; both agree with the
    oracle's SpMMV and filter."""
    A = O.anderson(12, 1.0, 5.0, 4)
    m_u = fd.build_matrix("csr", csr=(A.rowptr, A.col, A.val))
    # row 0: columns ascending with the diagonal; add column D-2 if absent
    cols0 = list(A.col[A.rowptr[0]:A.rowptr[1]])
    extra = next(c for c in range(A.D - 1, 0, -1) if c not in cols0)
    rp = A.rowptr.copy()
    rp[1:] += 1
    c0 = np.array(sorted(cols0 + [extra]), np.uint32)
    v0 = np.array([A.val[A.rowptr[0] + cols0.index(c)] if c in cols0 else 0.0 for c in c0])
    col = np.concatenate([c0, A.col[A.rowptr[1]:]])
    val = np.concatenate([v0, A.val[A.rowptr[1]:]])
    m_n = fd.build_matrix("csr", csr=(rp, col, val))
    X = dev(start_block(A.D, nb, 5))
    Yu, Yn = torch.empty_like(X), torch.empty_like(X)
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    mu = O.cheb_coeffs(1, beta, 0.0, 9)
    Vu, Vn = dev(start_block(A.D, nb, 6)), dev(start_block(A.D, nb, 6))
    W1, W2 = torch.empty_like(X), torch.empty_like(X)
    try:
        fd.spmmv_tune(0, 2, 1, 512, 1, 0, 0, shfl)
        fd.spmmv(m_u, X, Yu)
        fd.spmmv(m_n, X, Yn)
        fd.cheb_filter(m_u, Vu, mu, alpha, beta, W1, W2, nb)
        fd.cheb_filter(m_n, Vn, mu, alpha, beta, W1, W2, nb)
        torch.cuda.synchronize()
    finally:
        fd.spmmv_tune()
    assert torch.equal(Yu, Yn)
    assert torch.equal(Vu, Vn)
    assert relerr(Yu.cpu().numpy(), O.spmmv(A, start_block(A.D, nb, 5))) <= 1e-14
    assert relerr(Vu.cpu().numpy(), O.cheb_filter(A, start_block(A.D, nb, 6), mu, alpha, beta)) <= 1e-12
