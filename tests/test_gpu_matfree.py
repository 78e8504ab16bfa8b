"""GPU parity of the matrix-free Hubbard format (H = H_up x I + I x H_dn + U D
applied from per-species hop tables, no stored matrix) against the oracle's
stored Hubbard matrix, through the C ABI.

Tolerances as for the stored formats: FP64 within 1e-12 relative of the
oracle; bit-exact where every partial sum is an exact integer; FP32 filter
within the degree-times-unit-roundoff bound.  The down-state tile and the XCD
remap only reorder rows, never the arithmetic of a row: results are bitwise
equal across launch shapes.
"""
import numpy as np
import pytest

import oracle as O
from fd_inputs import int_block, start_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402

# (L, n_up, n_dn, t, U, periodic): square, unequal species, a single up state
# (n_up = 0), open chain, non-unit hopping
CASES = {
    "hub8": (8, 4, 4, 1.0, 4.0, True),
    "hub7": (7, 3, 2, 1.0, 2.5, True),
    "hub9": (9, 4, 5, 0.5, 8.0, True),
    "hub5_0": (5, 0, 2, 1.0, 1.0, True),
    "hub8_open": (8, 4, 4, 1.0, 4.0, False),
}


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def build(name, C_=0):
    L, nu, nd, t, U, per = CASES[name]
    m = fd.build_matrix("hubbard", fmt="matfree", C_=C_, L=L, n_up=nu, n_dn=nd, t=t, U=U, periodic=per)
    return m, O.hubbard(L, nu, nd, t, U, per)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nb", [1, 2, 4, 8, 16, 32, 64])
def test_matfree_spmmv_fp64_parity(name, nb):
    m, A = build(name)
    assert (m.D, m.nnz) == (A.D, int(A.rowptr[-1]))
    X = start_block(A.D, nb, 11)
    Y = torch.empty((A.D, nb), dtype=torch.float64, device="cuda")
    fd.spmmv(m, dev(X), Y)
    torch.cuda.synchronize()
    assert relerr(Y.cpu().numpy(), O.spmmv(A, X)) <= 1e-12


@pytest.mark.parametrize("name", ["hub8", "hub7", "hub8_open"])
@pytest.mark.parametrize("C_", [1, 3, 16, 1000])
@pytest.mark.parametrize("nb", [1, 8, 64])
def test_matfree_spmmv_integer_bit_exact(name, C_, nb):
    """Integer blocks: every partial sum is exact in FP64 (|x| < 2^10) and in
    FP32 (|x| < 2^8), so the result equals the oracle's bit for bit, whatever
    the tile C."""
    m, A = build(name, C_)
    for dt, bound in ((torch.float64, 1 << 10), (torch.float32, 1 << 8)):
        X = int_block(A.D, nb, 3, bound)
        Y = torch.empty((A.D, nb), dtype=dt, device="cuda")
        fd.spmmv(m, dev(X, dt), Y)
        torch.cuda.synchronize()
        assert np.array_equal(Y.cpu().double().numpy(), O.spmmv(A, X))


def test_matfree_spmmv_ld_and_errors():
    m, A = build("hub7")
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


@pytest.mark.parametrize("name", ["hub8", "hub9", "hub5_0"])
@pytest.mark.parametrize("nb,nbund,concurrent", [(1, 2, False), (8, 3, True), (16, 2, False), (64, 1, False)])
def test_matfree_filter_fp64_parity(name, nb, nbund, concurrent):
    """All fused step forms (first, second, general step) against the oracle's
    unfused three-term recurrence."""
    m, A = build(name)
    alpha, beta = O.scaling(*O.gershgorin(A))
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


def test_matfree_filter_fp32_error():
    m, A = build("hub8")
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(0, alpha * -0.5 + beta, alpha * 0.5 + beta, 100)
    V = start_block(A.D, 16, 6).astype(np.float32)
    Vd = dev(V)
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, 16)
    torch.cuda.synchronize()
    ref = O.cheb_filter(A, V.astype(np.float64), mu, alpha, beta)
    assert relerr(Vd.cpu().double().numpy(), ref) <= 100 * 2.0 ** -24 * 10


@pytest.mark.parametrize("xcd,nt,tile,wide,shfl,lds", [(1, 1, 0, 0, 2, 0), (0, 0, 1, 0, 2, 0), (1, 0, 5, 0, 2, 0),
                                                        (0, 1, 1000, 0, 2, 0), (1, 1, 2, 0, 2, 0), (0, 1, 64, 1, 2, 0),
                                                        (1, 1, 3, 1, 2, 0), (0, 1, 16, 0, 0, 0), (1, 0, 7, 1, 0, 0),
                                                        (1, 1, 0, 0, 2, 1), (0, 0, 5, 0, 1, 1), (0, 1, 16, 1, 2, 1),
                                                        (1, 1, 3, 0, 0, 1)])
def test_matfree_launch_shapes_bitwise_equal(xcd, nt, tile, wide, shfl, lds):
    """Tile, XCD remap, lane width, hop loop (permute or broadcast) and the
    LDS-staged down pass only change the order rows are visited in and
    where the gathered rows come from: bitwise equal results."""
    m, A = build("hub9")
    X = dev(start_block(A.D, 16, 1))
    Y0 = torch.empty_like(X)
    fd.spmmv(m, X, Y0)
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(0, -0.2, 0.2, 9)
    V0 = start_block(A.D, 32, 2)
    Va = dev(V0)
    W1 = torch.empty_like(Va)
    W2 = torch.empty_like(Va)
    fd.cheb_filter(m, Va, mu, alpha, beta, W1, W2, 16)
    try:
        fd.spmmv_tune(0, xcd, 1, 1024, nt, wide, tile, shfl, 0, lds)
        Y1 = torch.empty_like(X)
        fd.spmmv(m, X, Y1)
        Vb = dev(V0)
        fd.cheb_filter(m, Vb, mu, alpha, beta, W1, W2, 16)
        torch.cuda.synchronize()
    finally:
        fd.spmmv_tune()
    assert torch.equal(Y0, Y1)
    assert torch.equal(Va, Vb)


def test_matfree_autotune_keeps_results():
    m, A = build("hub8")
    X = dev(start_block(A.D, 8, 3))
    Y0 = torch.empty_like(X)
    fd.spmmv(m, X, Y0)
    shape = fd.autotune(m, "f64", 8)
    assert shape[1] in (0, 1) and shape[6] >= 1
    Y1 = torch.empty_like(X)
    fd.spmmv(m, X, Y1)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)


@pytest.mark.parametrize("name,nb,nmom", [("hub8", 16, 64), ("hub7", 1, 10)])
def test_matfree_kpm_moments_parity(name, nb, nmom):
    m, A = build(name)
    alpha, beta = O.scaling(*O.gershgorin(A))
    R = start_block(A.D, nb, 31)
    mu = fd.kpm_moments(m, dev(R), nmom, alpha, beta)
    ref = O.kpm_moments(A, R, nmom, alpha, beta)
    assert np.abs(mu - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_matfree_hubbard8_solve_vs_dense(precision):
    """fd_solve on the matrix-free form: Hubbard L=8 (4+4, U=4), 16 pairs
    nearest 0 in [-0.5, 0.5], the same run as for the stored formats."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = np.linalg.eigvalsh(A.dense())
    inside = ev[(ev >= -0.5) & (ev <= 0.5)]
    want = np.sort(inside[np.argsort(np.abs(inside), kind="stable")[:16]])
    m, _ = build("hub8")
    r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, precision=precision,
                 V0=start_block(A.D, 128, 0))
    assert r.status == fd.FD_OK, r.stats
    normH = r.stats["norm_H"]
    assert np.abs(r.evals - want).max() <= 1e-10 * normH
    X = r.evecs.cpu().numpy()
    assert np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0).max() <= 1e-9 * normH
