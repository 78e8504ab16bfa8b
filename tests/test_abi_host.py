"""libfd without a GPU: the shared library loads and exports every entry point
that include/fd.h declares; the host-side builders match the oracle bit for
bit; coefficients agree; argument errors follow the documented conventions."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2209_01974_amd as fd
from lattice_walk import permuted_csr, tile_walk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(fd.LIB_PATH):
        from paper_2209_01974_amd import build
        build.build()


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "fd.h")).read()
    declared = set(re.findall(r"^\s*(?:fd_status|void|int32_t|const char \*)\s*(fd_[a-z_]+)\s*\(", hdr, re.M))
    assert {"fd_build_matrix", "fd_spmmv", "fd_cheb_filter", "fd_orthog", "fd_rayleigh_ritz",
            "fd_solve"} <= declared
    L = fd.lib()
    for name in declared:
        assert hasattr(L, name), name


def _same_csr(m, A):
    rowptr, col, val = m.export_csr()
    assert np.array_equal(rowptr, A.rowptr)
    assert np.array_equal(col, A.col)
    assert np.array_equal(val.view(np.uint64), A.val.view(np.uint64))


@pytest.mark.parametrize("L,nu,nd,U,per", [(6, 3, 3, 4.0, True), (8, 4, 4, 4.0, True), (7, 2, 3, 2.5, True),
                                           (8, 4, 4, 4.0, False), (5, 0, 2, 1.0, True), (6, 3, 3, 0.0, True)])
def test_hubbard_bit_exact(L, nu, nd, U, per):
    m = fd.build_matrix("hubbard", host_only=True, L=L, n_up=nu, n_dn=nd, t=1.0, U=U, periodic=per)
    _same_csr(m, O.hubbard(L, nu, nd, 1.0, U, per))


def test_hubbard_zero_hopping_stores_diagonal_only():
    m = fd.build_matrix("hubbard", host_only=True, L=6, n_up=3, n_dn=3, t=0.0, U=2.0)
    _same_csr(m, O.hubbard(6, 3, 3, 0.0, 2.0))
    assert m.nnz == m.D


@pytest.mark.parametrize("L,W,seed", [(3, 16.5, 1), (5, 16.5, 1), (12, 3.0, 7)])
def test_anderson_bit_exact(L, W, seed):
    m = fd.build_matrix("anderson", host_only=True, L=L, t=1.0, W=W, seed=seed)
    _same_csr(m, O.anderson(L, 1.0, W, seed))


@pytest.mark.slow
def test_hubbard_config_sizes_and_gershgorin():
    m = fd.build_matrix("hubbard", host_only=True, L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    assert (m.D, m.nnz) == (4900, 49700)
    assert (m.lam_lo, m.lam_hi) == O.gershgorin(O.hubbard(8, 4, 4, 1.0, 4.0))
    m = fd.build_matrix("anderson", host_only=True, L=40, t=1.0, W=16.5, seed=1)
    A = O.anderson(40, 1.0, 16.5, 1)
    _same_csr(m, A)
    assert (m.lam_lo, m.lam_hi) == O.gershgorin(A)


@pytest.mark.parametrize("C_,sigma", [(1, 1), (4, 1), (8, 32), (32, 128), (64, 1 << 20)])
def test_sell_bit_exact(C_, sigma):
    m = fd.build_matrix("hubbard", fmt="sell", C_=C_, sigma=sigma, host_only=True, L=7, n_up=3, n_dn=2,
                        t=1.0, U=3.0)
    S = O.sell(O.hubbard(7, 3, 2, 1.0, 3.0), C_, sigma)
    perm, cptr, clen, col, val = m.export_sell()
    assert np.array_equal(perm, S.perm)
    assert np.array_equal(cptr, S.chunk_ptr)
    assert np.array_equal(clen, S.chunk_len)
    assert np.array_equal(col, S.col)
    assert np.array_equal(val.view(np.uint64), S.val.view(np.uint64))


def test_sell_round_trip_to_csr():
    A = O.anderson(6, 1.0, 5.0, 2)
    m = fd.build_matrix("anderson", fmt="sell", C_=16, sigma=64, host_only=True, L=6, t=1.0, W=5.0, seed=2)
    perm, cptr, clen, col, val = m.export_sell()
    C_ = 16
    for s in range(A.D):
        o = perm[s]
        c, r = divmod(s, C_)
        n = A.rowptr[o + 1] - A.rowptr[o]
        got_c = [col[cptr[c] + j * C_ + r] for j in range(n)]
        got_v = [val[cptr[c] + j * C_ + r] for j in range(n)]
        assert got_c == list(A.col[A.rowptr[o]:A.rowptr[o + 1]])
        assert got_v == list(A.val[A.rowptr[o]:A.rowptr[o + 1]])


def test_user_csr_and_diagonal_round_trip():
    A = O.hubbard(6, 2, 3, 1.0, 1.5)
    m = fd.build_matrix("csr", host_only=True, csr=(A.rowptr, A.col, A.val))
    _same_csr(m, A)
    d = np.linspace(-1, 1, 17)
    m = fd.build_matrix("diagonal", host_only=True, diag=d)
    _same_csr(m, O.diagonal(d))


def test_user_csr_rejects_bad_input():
    A = O.hubbard(6, 2, 3, 1.0, 1.5)
    col = A.col.copy()
    col[1], col[2] = col[2], col[1]
    with pytest.raises(fd.FDError) as e:
        fd.build_matrix("csr", host_only=True, csr=(A.rowptr, col, A.val))
    assert e.value.status == fd.FD_ERR_INVALID


@pytest.mark.parametrize("kind,a,b,n", [(0, -0.3, 0.2, 50), (0, -1.0, 1.0, 10), (1, 0.1, 0.0, 800),
                                        (0, 0.01, 0.02, 800)])
def test_coefficients_match_oracle(kind, a, b, n):
    np.testing.assert_allclose(fd.cheb_coeffs(kind, a, b, n), O.cheb_coeffs(kind, a, b, n), rtol=0, atol=2e-15)


def test_argument_errors():
    with pytest.raises(fd.FDError) as e:
        fd.build_matrix("hubbard", host_only=True, L=2, n_up=1, n_dn=1)
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError) as e:
        fd.build_matrix("anderson", fmt="sell", C_=3, sigma=1, host_only=True, L=4)
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError):
        fd.cheb_coeffs(0, 0.5, 0.2, 10)
    # device entry points refuse a host-only matrix before touching the GPU
    m = fd.build_matrix("anderson", host_only=True, L=4, W=1.0)
    st = fd.lib().fd_spmmv(m.handle, fd.FD_F64, 8, C.c_void_p(256), 8, C.c_void_p(1 << 20), 8, None)
    assert st == fd.FD_ERR_INVALID
    assert b"host-only" in fd.lib().fd_last_error()
    st = fd.lib().fd_orthog(10, 0, None, 1, 0, 0, None, None)
    assert st == fd.FD_ERR_INVALID


@pytest.mark.parametrize("L,nu,nd,U,t,per", [(6, 3, 3, 4.0, 1.0, True), (8, 4, 4, 4.0, 1.0, True),
                                             (7, 2, 3, 2.5, 1.0, True), (8, 4, 4, 4.0, 1.0, False),
                                             (5, 0, 2, 1.0, 1.0, True), (6, 3, 3, 2.0, 0.0, True),
                                             (9, 4, 5, 8.0, 0.5, True)])
def test_matfree_sizes_and_gershgorin_match_csr(L, nu, nd, U, t, per):
    """The tensor-product (matrix-free) form describes the same matrix: the
    same dimension and non-zero count as the stored Hubbard matrix, and the
    same Gershgorin interval as the oracle's CSR (exact: row sums of +-t and
    an integer multiple of U)."""
    m = fd.build_matrix("hubbard", fmt="matfree", host_only=True, L=L, n_up=nu, n_dn=nd, t=t, U=U, periodic=per)
    A = O.hubbard(L, nu, nd, t, U, per)
    assert (m.D, m.nnz) == (A.D, int(A.rowptr[-1]))
    assert (m.lam_lo, m.lam_hi) == O.gershgorin(A)
    with pytest.raises(fd.FDError):
        m.export_csr()


def test_matfree_argument_errors():
    with pytest.raises(fd.FDError) as e:
        fd.build_matrix("anderson", fmt="matfree", host_only=True, L=4, W=1.0)
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError) as e:
        fd.build_matrix("hubbard", fmt="matfree", C_=-1, host_only=True, L=6, n_up=3, n_dn=3)
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError):
        fd.spmmv_tune(tile=-1)
    for bad in (-1, 3):
        with pytest.raises(fd.FDError):
            fd.spmmv_tune(shfl=bad)
    fd.spmmv_tune()


def test_anderson_stream_offset_bit_exact():
    """skip = k: the disorder continues after k draws of the stream.  The
    oracle's diagonal is W (u_{i+k} - 1/2) of its own SplitMix64 stream, and
    the library's counter-based draw gives the same bits."""
    L, W, seed, k = 5, 7.5, 123, 2
    A = O.anderson(L, 1.0, W, seed, skip=k)
    u = O.uniforms(seed, L ** 3 + k)
    diag = np.array([A.val[A.rowptr[i]:A.rowptr[i + 1]][A.col[A.rowptr[i]:A.rowptr[i + 1]] == i][0]
                     for i in range(A.D)])
    assert np.array_equal(diag, W * (u[k:] - 0.5))
    m = fd.build_matrix("anderson", host_only=True, L=L, t=1.0, W=W, seed=seed, skip=k)
    _same_csr(m, A)


def test_anderson_batch_instance_draws():
    """Instance parameters come from the first two draws of SplitMix64(s),
    the same generator as the oracle's (two implementations)."""
    from fd_inputs import _splitmix64_uniforms, anderson_batch
    for s in (0, 100, 195, 2 ** 63 + 5):
        assert np.array_equal(np.array(_splitmix64_uniforms(s, 4)), O.uniforms(s, 4))
    inst = anderson_batch(range(100, 196))
    assert len(inst) == 96
    assert all(20 <= q["L"] <= 64 and 2.0 <= q["W"] < 20.0 and q["skip"] == 2 for q in inst)


@pytest.mark.parametrize("L,tx,ty", [(6, 4, 3), (5, 2, 2), (6, 1, 1), (5, 9, 2), (7, 7, 7)])
def test_anderson_tiled_numbering_is_the_permuted_matrix(L, tx, ty):
    """Tiled site numbering: the matrix is P A P^T of the naturally numbered
    oracle matrix, bit for bit; one tile over the whole (x, y) plane walks
    the natural order itself."""
    A = O.anderson(L, 1.0, 6.0, 3)
    p = tile_walk(L, tx, ty)
    assert np.array_equal(p, [x + L * y + L * L * z for y0 in range(0, L, ty) for x0 in range(0, L, tx)
                              for z in range(L) for y in range(y0, min(L, y0 + ty))
                              for x in range(x0, min(L, x0 + tx))])
    assert np.array_equal(np.sort(p), np.arange(A.D))
    m = fd.build_matrix("anderson", host_only=True, L=L, t=1.0, W=6.0, seed=3, tiles=(tx, ty))
    _same_csr(m, permuted_csr(A, p))
    if tx >= L and ty >= L:
        assert np.array_equal(p, np.arange(A.D))
        _same_csr(m, A)


def test_anderson_tiled_numbering_argument_errors():
    for tiles in ((3, 0), (0, 2), (-1, -1)):
        with pytest.raises(fd.FDError) as e:
            fd.build_matrix("anderson", host_only=True, L=5, t=1.0, W=1.0, tiles=tiles)
        assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError):
        fd.build_matrix("anderson", fmt="pencil", C_=2, sigma=2, host_only=True, L=5, t=1.0, W=1.0, tiles=(2, 2))


def test_pencil_order_is_the_csr_in_a_lattice_walk():
    """Pencil-ordered Anderson: perm walks (x, y) tiles over all z; every
    stored row is the CSR row it names, unpadded (SELL-1)."""
    A = O.anderson(5, 1.0, 4.0, 2)
    m = fd.build_matrix("anderson", fmt="pencil", C_=2, sigma=3, host_only=True, L=5, t=1.0, W=4.0, seed=2)
    perm, cptr, clen, col, val = m.export_sell()
    assert np.array_equal(np.sort(perm), np.arange(A.D))
    L = 5
    want = [x + L * y + L * L * z for y0 in range(0, L, 3) for x0 in range(0, L, 2) for z in range(L)
            for y in range(y0, min(L, y0 + 3)) for x in range(x0, min(L, x0 + 2))]
    assert np.array_equal(perm, want)
    for r, o in enumerate(perm):
        a, b = A.rowptr[o], A.rowptr[o + 1]
        assert clen[r] == b - a
        assert np.array_equal(col[cptr[r]:cptr[r + 1]], A.col[a:b])
        assert np.array_equal(val[cptr[r]:cptr[r + 1]], A.val[a:b])
    with pytest.raises(fd.FDError):
        fd.build_matrix("hubbard", fmt="pencil", host_only=True, L=6, n_up=3, n_dn=3)


@pytest.mark.parametrize("L,nu,nd,U,per", [(8, 4, 4, 4.0, True), (7, 2, 3, 2.5, True), (8, 4, 3, 1.0, False)])
def test_hubbard_rcm_labels_are_a_relabeling(L, nu, nd, U, per):
    """config_order 1: the library's matrix is P A P^T of the oracle's ranked
    one, bit for bit, with P read from the exported configurations (each
    label's spin configuration, mapped to its oracle rank); and labels one
    hop apart are close (the bandwidth of a species' hop graph shrinks)."""
    import math
    m = fd.build_matrix("hubbard", host_only=True, L=L, n_up=nu, n_dn=nd, t=1.0, U=U, periodic=per,
                        config_order=1)
    cu, cd = math.comb(L, nu), math.comb(L, nd)
    up, dn = m.export_configs(cu, cd)
    rank_u = {x: i for i, x in enumerate(x for x in range(1 << L) if bin(x).count("1") == nu)}
    rank_d = {x: i for i, x in enumerate(x for x in range(1 << L) if bin(x).count("1") == nd)}
    pu = np.array([rank_u[int(x)] for x in up])
    pd = np.array([rank_d[int(x)] for x in dn])
    assert sorted(pu) == list(range(cu)) and sorted(pd) == list(range(cd))
    P = (pu[:, None] * cd + pd[None, :]).ravel()  # label row -> oracle row
    A = O.hubbard(L, nu, nd, 1.0, U, per)
    rowptr, col, val = m.export_csr()
    Ad = A.dense()
    import scipy.sparse as sp
    Ml = sp.csr_matrix((val, col, rowptr), shape=(m.D, m.D)).toarray()
    assert np.array_equal(Ml.view(np.uint64), Ad[np.ix_(P, P)].view(np.uint64))
    # canonical CSR: ascending columns, diagonal stored
    for i in range(m.D):
        c = col[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(c.astype(np.int64)) > 0) and i in c
    # the ranked basis exports its configurations in rank order
    m0 = fd.build_matrix("hubbard", host_only=True, L=L, n_up=nu, n_dn=nd, t=1.0, U=U, periodic=per)
    up0, dn0 = m0.export_configs(cu, cd)
    assert [rank_u[int(x)] for x in up0] == list(range(cu))


def test_hubbard14_rcm_labels_shrink_up_hop_distance():
    """Hubbard L=14 (7+7): in the ranked basis an up hop moves up to 1,912
    slabs of 3,432 rows; with reverse Cuthill-McKee labels at most 369."""
    for order, bound in ((0, 1912), (1, 369)):
        m = fd.build_matrix("hubbard", host_only=True, L=14, n_up=7, n_dn=7, t=1.0, U=8.0, config_order=order)
        rowptr, col, _ = m.export_csr()
        rows = np.repeat(np.arange(m.D, dtype=np.int64), np.diff(rowptr))
        assert (np.abs(col.astype(np.int64) - rows) // 3432).max() == bound
        del rowptr, col, rows
        m.free()


def test_kpm_count_host_call():
    """fd_kpm_count on exact-trace moments (oracle, Anderson L=5): the
    Jackson-damped count of a window matches the dense eigenvalue count to
    within the kernel's broadening, and feeding damped moments with kind 2
    gives the same number as plain moments with kind 0; mu_0 <= 0 is
    rejected."""
    A = O.anderson(5, 1.0, 4.0, 3)
    lam = np.linalg.eigvalsh(A.dense())
    lo, hi = O.gershgorin(A)
    alpha, beta = O.scaling(lo, hi)
    nmom = 600
    mu = O.kpm_moments(A, np.sqrt(A.D) * np.eye(A.D), nmom, alpha, beta)
    for wl, wh in ((-1.0, 1.0), (-3.0, 0.5), (2.0, 6.0)):
        a, b = alpha * wl + beta, alpha * wh + beta
        est = fd.window_count(mu, A.D, a, b)
        true = np.sum((lam >= wl) & (lam <= wh))
        assert abs(est - true) <= 2.0, (wl, wh, est, true)
        g = np.array([O.jackson(nmom - 1, k) for k in range(nmom)])
        est2 = fd.window_count(g * mu, A.D, a, b, damped=True)
        assert abs(est2 - est) <= 1e-12 * A.D
    with pytest.raises(fd.FDError) as e:
        fd.window_count(np.zeros(8), 10, -0.5, 0.5)
    assert e.value.status == fd.FD_ERR_INVALID


@pytest.mark.slow
@pytest.mark.parametrize("model", ["anderson200", "hubbard14"])
def test_full_size_matrices_bit_exact(model):
    """The two full-size matrices the benchmarks run, exported from the
    library's host builder, equal the oracle's CSR bit for bit: Anderson
    L=200 (W=16.5, seed 1; D = 8,000,000) and the Hubbard ring L=14 (7+7,
    U=8, ranked basis; D = 11,778,624)."""
    if model == "anderson200":
        m = fd.build_matrix("anderson", host_only=True, L=200, t=1.0, W=16.5, seed=1)
        A = O.anderson(200, 1.0, 16.5, 1)
    else:
        m = fd.build_matrix("hubbard", host_only=True, L=14, n_up=7, n_dn=7, t=1.0, U=8.0)
        A = O.hubbard(14, 7, 7, 1.0, 8.0)
    assert (m.D, m.nnz) == (A.D, A.nnz)
    _same_csr(m, A)
    m.free()
