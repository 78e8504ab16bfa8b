"""GPU parity of the batched path (many instances stacked as one
block-diagonal matrix, per-instance scaling, coefficients and degree, one
launch per degree step, optionally replayed from a HIP graph) against the
oracle run instance by instance.

Tolerances as for single matrices: FP64 within 1e-12 relative per instance;
bit-exact for integer blocks; idle instances unchanged bit for bit; graph
replays bitwise equal to the eager launches (same kernels, same order).
"""
import numpy as np
import pytest

import oracle as O
from fd_inputs import int_block, start_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402

# uneven instances: Anderson of several sizes and disorders (one built from
# a stream offset), Hubbard rings, one stored as SELL
INST = [
    (dict(model="anderson", L=5, t=1.0, W=4.0, seed=3), lambda: O.anderson(5, 1.0, 4.0, 3)),
    (dict(model="hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0), lambda: O.hubbard(6, 3, 3, 1.0, 4.0)),
    (dict(model="anderson", L=7, t=1.0, W=16.5, seed=1, skip=2), lambda: O.anderson(7, 1.0, 16.5, 1, skip=2)),
    (dict(model="hubbard", L=7, n_up=3, n_dn=2, t=1.0, U=2.5, fmt="sell", C_=8, sigma=64),
     lambda: O.hubbard(7, 3, 2, 1.0, 2.5)),
    (dict(model="anderson", L=9, t=1.0, W=10.0, seed=5), lambda: O.anderson(9, 1.0, 10.0, 5)),
]


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def batch():
    mats = [fd.build_matrix(**kw) for kw, _ in INST]
    As = [ora() for _, ora in INST]
    b = fd.Batch(mats)
    del mats  # the batch keeps its own copy
    assert b.D == sum(A.D for A in As)
    assert np.array_equal(np.diff(b.off), [A.D for A in As])
    return b, As


@pytest.mark.parametrize("nb", [1, 4, 8, 16, 64])
def test_batch_spmmv_fp64_parity(batch, nb):
    b, As = batch
    X = start_block(b.D, nb, 7)
    Y = torch.empty((b.D, nb), dtype=torch.float64, device="cuda")
    fd.batch_spmmv(b, dev(X), Y)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    for i, A in enumerate(As):
        r = slice(b.off[i], b.off[i + 1])
        assert relerr(Yh[r], O.spmmv(A, X[r])) <= 1e-12


@pytest.mark.parametrize("nb", [1, 8, 64])
def test_batch_spmmv_integer_bit_exact(nb):
    kws = [dict(model="anderson", L=6, t=1.0, W=0.0, seed=1), dict(model="hubbard", L=6, n_up=3, n_dn=3, t=1.0,
                                                                   U=4.0),
           dict(model="anderson", L=4, t=1.0, W=0.0, seed=1)]
    As = [O.anderson(6, 1.0, 0.0, 1), O.hubbard(6, 3, 3, 1.0, 4.0), O.anderson(4, 1.0, 0.0, 1)]
    b = fd.Batch([fd.build_matrix(**kw) for kw in kws])
    for dt, bound in ((torch.float64, 1 << 10), (torch.float32, 1 << 8)):
        X = int_block(b.D, nb, 4, bound)
        Y = torch.empty((b.D, nb), dtype=dt, device="cuda")
        fd.batch_spmmv(b, dev(X, dt), Y)
        torch.cuda.synchronize()
        Yh = Y.cpu().double().numpy()
        for i, A in enumerate(As):
            r = slice(b.off[i], b.off[i + 1])
            assert np.array_equal(Yh[r], O.spmmv(A, X[r]))


def _filter_setup(b, As, degrees, seed):
    """Per-instance alpha, beta (Gershgorin) and coefficients: the indicator
    of a window around the middle of the spectrum, or the damped delta."""
    alpha, beta, mu = [], [], []
    for i, A in enumerate(As):
        lo, hi = O.gershgorin(A)
        a, c = O.scaling(lo, hi)
        alpha.append(a)
        beta.append(c)
        n = degrees[i]
        if n == 0:
            mu.append(np.zeros(1))
        elif i % 2:
            mu.append(O.cheb_coeffs(1, a * (0.5 * (lo + hi)) + c, 0.0, n))
        else:
            mid, w = 0.5 * (lo + hi), 0.1 * (hi - lo)
            mu.append(O.cheb_coeffs(0, a * (mid - w) + c, a * (mid + w) + c, n))
    return alpha, beta, mu


@pytest.mark.parametrize("nb,nbund", [(1, 2), (8, 3), (16, 2), (64, 1)])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_filter_fp64_parity(batch, nb, nbund, use_graph):
    """Uneven degrees, one idle instance (degree 0, left bit for bit)."""
    b, As = batch
    degrees = [23, 7, 0, 2, 40]
    alpha, beta, mu = _filter_setup(b, As, degrees, 0)
    ns = nb * nbund
    V = start_block(b.D, ns, 3)
    Vd = dev(V)
    W1 = torch.empty((b.D, ns), dtype=torch.float64, device="cuda")
    W2 = torch.empty_like(W1)
    fd.batch_filter(b, Vd, mu, degrees, alpha, beta, W1, W2, nb, use_graph=use_graph)
    torch.cuda.synchronize()
    got = Vd.cpu().numpy()
    for i, A in enumerate(As):
        r = slice(b.off[i], b.off[i + 1])
        if degrees[i] == 0:
            assert np.array_equal(got[r], V[r])
        else:
            ref = O.cheb_filter(A, V[r], mu[i], alpha[i], beta[i])
            assert relerr(got[r], ref) <= 1e-12


def test_batch_filter_fp32_error(batch):
    b, As = batch
    degrees = [30, 30, 30, 30, 30]
    alpha, beta, mu = _filter_setup(b, As, degrees, 0)
    V = start_block(b.D, 16, 6).astype(np.float32)
    Vd = dev(V)
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.batch_filter(b, Vd, mu, degrees, alpha, beta, W1, W2, 16, use_graph=True)
    torch.cuda.synchronize()
    got = Vd.cpu().double().numpy()
    for i, A in enumerate(As):
        r = slice(b.off[i], b.off[i + 1])
        ref = O.cheb_filter(A, V[r].astype(np.float64), mu[i], alpha[i], beta[i])
        assert relerr(got[r], ref) <= 30 * 2.0 ** -24 * 10


def test_batch_graph_replays_match_eager(batch):
    """One captured graph, replayed several times with eager work (copies,
    other kernels) and synchronizations in between, and with the
    per-instance degrees and coefficients changed between replays (they are
    read from device memory at run time): every replay equals the eager
    launches bit for bit."""
    b, As = batch
    nb, ns = 8, 16
    V0 = dev(start_block(b.D, ns, 9))
    V = torch.empty_like(V0)
    W1 = torch.empty_like(V0)
    W2 = torch.empty_like(V0)
    X = dev(start_block(b.D, nb, 10))
    Y = torch.empty_like(X)
    for rep, degrees in enumerate(([31, 12, 31, 5, 20], [31, 12, 31, 5, 20], [4, 31, 0, 31, 2],
                                   [31, 31, 31, 31, 31])):
        alpha, beta, mu = _filter_setup(b, As, degrees, rep)
        # eager reference
        V.copy_(V0)
        fd.batch_filter(b, V, mu, degrees, alpha, beta, W1, W2, nb, use_graph=False)
        ref = V.clone()
        fd.batch_spmmv(b, X, Y)  # unrelated eager work between the runs
        torch.cuda.synchronize()
        V.copy_(V0)
        fd.batch_filter(b, V, mu, degrees, alpha, beta, W1, W2, nb, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(V, ref), rep


def test_batch_errors():
    m = fd.build_matrix("anderson", L=4, W=1.0)
    mf = fd.build_matrix("hubbard", fmt="matfree", L=6, n_up=3, n_dn=3, U=4.0)
    with pytest.raises(fd.FDError):
        fd.Batch([m, mf])
    b = fd.Batch([m])
    V = torch.zeros((b.D, 8), dtype=torch.float64, device="cuda")
    W1 = torch.zeros_like(V)
    with pytest.raises(fd.FDError):  # W1 == W2
        fd.batch_filter(b, V, [np.ones(5)], [4], [0.1], [0.0], W1, W1, 8)
    with pytest.raises(fd.FDError):  # degree 1
        fd.batch_filter(b, V, [np.ones(2)], [1], [0.1], [0.0], W1, torch.zeros_like(V), 8)


@pytest.mark.parametrize("ortho,ns", [(fd.FD_ORTHO_SVQB2, 64), (fd.FD_ORTHO_CHOLQR2, 64), (fd.FD_ORTHO_SVQB2, 128)])
def test_solve_batch_vs_dense_and_single(ortho, ns):
    """Five uneven instances, 8 pairs nearest tau each (damped delta at
    tau, or a window), nb = 16: every instance's eigenvalues match its dense
    spectrum and the single-instance fd_solve on the same start block;
    residuals recomputed from the returned vectors.  N_s = 64 runs the
    dense steps of all instances at once (batched Gram, Cholesky, Jacobi
    eigensolve, rotations, residuals); N_s = 128 runs them one by one."""
    kws = [dict(model="anderson", L=8, t=1.0, W=5.0, seed=2), dict(model="anderson", L=10, t=1.0, W=16.5, seed=1),
           dict(model="hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0),
           dict(model="anderson", L=9, t=1.0, W=12.0, seed=7, skip=2),
           dict(model="hubbard", L=7, n_up=3, n_dn=3, t=1.0, U=3.0)]
    As = [O.anderson(8, 1.0, 5.0, 2), O.anderson(10, 1.0, 16.5, 1), O.hubbard(6, 3, 3, 1.0, 4.0),
          O.anderson(9, 1.0, 12.0, 7, skip=2), O.hubbard(7, 3, 3, 1.0, 3.0)]
    windows = [(0.0, 0.0), (0.5, 0.5), (-0.5, 0.45), (0.0, 0.0), (-1.0, 1.0)]
    degrees = [300, 300, 100, 300, 300]
    adapt = [0, 0, 0, 0, 1]  # [-1, 1] holds 167 eigenvalues of the last: track the window
    mats = [fd.build_matrix(**kw) for kw in kws]
    b = fd.Batch(mats)
    V0 = start_block(b.D, ns, 11)
    params = [dict(tau_lo=w[0], tau_hi=w[1], n_target=8, n_search=ns, nb=16, degree=d, max_iter=100, tol=1e-9,
                   adapt=a, ortho=ortho) for w, d, a in zip(windows, degrees, adapt)]
    r = fd.solve_batch(b, params, V0=V0, want_vectors=True)
    assert r.status == fd.FD_OK, (r.bstats, r.stats)
    assert r.bstats["n_converged"] == 5 and r.bstats["graph_launches"] >= 1
    X = r.evecs.cpu().numpy()
    for i, A in enumerate(As):
        ev = np.linalg.eigvalsh(A.dense())
        lo, hi = windows[i]
        tau = 0.5 * (lo + hi)
        pool = ev if hi <= lo else ev[(ev >= lo) & (ev <= hi)]
        want = np.sort(pool[np.argsort(np.abs(pool - tau), kind="stable")[:8]])
        normH = r.stats[i]["norm_H"]
        assert np.abs(r.evals[i] - want).max() <= 1e-10 * normH, i
        rows = slice(b.off[i], b.off[i + 1])
        Xi = X[rows]
        assert np.linalg.norm(O.spmmv(A, Xi) - Xi * r.evals[i], axis=0).max() <= 1e-9 * normH
        single = fd.solve(mats[i], lo, hi, 8, ns, 16, degrees[i], max_iter=100, tol=1e-9, V0=V0[rows],
                          want_vectors=False, adapt=adapt[i], ortho=ortho)
        assert single.status == fd.FD_OK
        assert np.abs(single.evals - r.evals[i]).max() <= 1e-10 * normH
        assert abs(single.stats["iters"] - r.stats[i]["iters"]) <= 1


@pytest.mark.parametrize("ortho", [fd.FD_ORTHO_SVQB2, fd.FD_ORTHO_CHOLQR2])
def test_solve_batch_rank_deficient_start_block(ortho):
    """One instance starts from a block with repeated columns: the batched
    orthogonalization sees the deficient rank (SVQB) or a failed Cholesky
    pivot, hands that instance to the one-by-one SVQB2 with refill, and the
    batch still converges to the dense answer."""
    kws = [dict(model="anderson", L=8, t=1.0, W=5.0, seed=2), dict(model="hubbard", L=6, n_up=3, n_dn=3, t=1.0, U=4.0),
           dict(model="anderson", L=9, t=1.0, W=12.0, seed=7, skip=2)]
    As = [O.anderson(8, 1.0, 5.0, 2), O.hubbard(6, 3, 3, 1.0, 4.0), O.anderson(9, 1.0, 12.0, 7, skip=2)]
    windows = [(0.0, 0.0), (-0.5, 0.45), (0.0, 0.0)]
    b = fd.Batch([fd.build_matrix(**kw) for kw in kws])
    V0 = start_block(b.D, 64, 5)
    r1 = slice(b.off[1], b.off[2])
    V0[r1, 32:] = V0[r1, :32]
    params = [dict(tau_lo=w[0], tau_hi=w[1], n_target=8, n_search=64, nb=16, degree=d, max_iter=100, tol=1e-9,
                   ortho=ortho) for w, d in zip(windows, (300, 100, 300))]
    r = fd.solve_batch(b, params, V0=V0)
    assert r.status == fd.FD_OK, (r.bstats, r.stats)
    for i, A in enumerate(As):
        ev = np.linalg.eigvalsh(A.dense())
        lo, hi = windows[i]
        tau = 0.5 * (lo + hi)
        pool = ev if hi <= lo else ev[(ev >= lo) & (ev <= hi)]
        want = np.sort(pool[np.argsort(np.abs(pool - tau), kind="stable")[:8]])
        assert np.abs(r.evals[i] - want).max() <= 1e-10 * r.stats[i]["norm_H"], i


def test_batch_autotune_keeps_results_bitwise(batch):
    """The batched autotuner only chooses the XCD chunk and the permute
    round width, which do not change how a row is summed: the filter is
    bitwise equal before and after tuning, and the chosen shape is one of
    the candidates."""
    b, As = batch
    degrees = [23, 7, 0, 2, 40]
    alpha, beta, mu = _filter_setup(b, As, degrees, 0)
    V = start_block(b.D, 32, 3)
    outs = []
    for tune in (False, True):
        if tune:
            nb, chunk, sh = fd.batch_autotune(b, "f64", 16)
            assert nb == 16 and chunk in (256, 512, 1024, 2048, 4096, 8192, 16384) and sh in (1, 2)
        Vd = dev(V)
        W1 = torch.empty_like(Vd)
        W2 = torch.empty_like(Vd)
        fd.batch_filter(b, Vd, mu, degrees, alpha, beta, W1, W2, 16)
        torch.cuda.synchronize()
        outs.append(Vd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    nb, _, _ = fd.batch_autotune(b, "f64", 0)
    assert nb in (8, 16, 32, 64)


def test_solve_batch_picks_the_bundle_width():
    """params nb = 0: the library times the batched step for the widths
    that divide N_s and uses the fastest; the answer is the one of nb = 16."""
    kws = [dict(model="anderson", L=8, t=1.0, W=5.0, seed=2), dict(model="hubbard", L=6, n_up=3, n_dn=3, t=1.0,
                                                                 U=4.0)]
    mats = [fd.build_matrix(**kw) for kw in kws]
    b = fd.Batch(mats)
    V0 = start_block(b.D, 64, 11)
    res = {}
    for nb in (16, 0):
        params = [dict(tau_lo=0.0, tau_hi=0.0, n_target=8, n_search=64, nb=nb, degree=300, max_iter=100, tol=1e-9)
                  for _ in kws]
        res[nb] = fd.solve_batch(b, params, V0=V0)
        assert res[nb].status == fd.FD_OK
    assert res[0].bstats["nb"] in (8, 16, 32, 64) and res[16].bstats["nb"] == 16
    for i in range(2):
        assert np.abs(res[0].evals[i] - res[16].evals[i]).max() <= 1e-10 * res[16].stats[i]["norm_H"]
