"""Pins for the oracle's generators and matrix builders (CPU only).

Each test checks the oracle against something other than itself: printed
values of the paper, published generator outputs, exact counting formulas,
closed-form spectra, or symmetries of the physics.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(path):
    with open(path) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_splitmix64_published_vector():
    want = [int(r[0], 16) for r in _rows(os.path.join(GOLD, "splitmix64_seed0.txt"))]
    assert O.splitmix64_first(0, 3) == want


def test_uniforms_range_and_mean():
    u = O.uniforms(1, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    # top 53 bits of each raw output, scaled by 2^-53
    raw = O.splitmix64_first(1, 4)
    np.testing.assert_array_equal(u[:4], [(r >> 11) * 2.0 ** -53 for r in raw])


@pytest.mark.parametrize("L,N", [(3, 1), (6, 2), (6, 3), (7, 3), (8, 4), (10, 5), (14, 7)])
def test_hubbard_counts_closed_form(L, N):
    # D = C(L,N)^2 ; nnz = D + 2 * [L * 2 C(L-2, N-1)] * C(L, N) on a ring
    D = math.comb(L, N) ** 2
    nnz = D + 2 * (L * 2 * math.comb(L - 2, N - 1)) * math.comb(L, N)
    import ctypes as C
    d, z = C.c_int64(), C.c_int64()
    assert O.lib().orc_hubbard_size(L, N, N, 1, 1.0, C.byref(d), C.byref(z)) == 0
    assert (d.value, z.value) == (D, nnz)


def test_hubbard_config_sizes():
    import ctypes as C
    d, z = C.c_int64(), C.c_int64()
    O.lib().orc_hubbard_size(8, 4, 4, 1, 1.0, C.byref(d), C.byref(z))
    assert (d.value, z.value) == (4900, 49700)
    O.lib().orc_hubbard_size(14, 7, 7, 1, 1.0, C.byref(d), C.byref(z))
    assert (d.value, z.value) == (11778624, 189364032)


def test_hubbard_paper_table2_open_chain():
    """Table 2 prints D and n_nzr for Hubbard14/16; the open chain without the
    stored diagonal reproduces both exactly."""
    import ctypes as C
    for L, N, D, nnzr in _rows(os.path.join(GOLD, "hubbard_table2.txt")):
        L, N, D, nnzr = int(L), int(N), int(D), float(nnzr)
        d, z = C.c_int64(), C.c_int64()
        O.lib().orc_hubbard_size(L, N, N, 0, 1.0, C.byref(d), C.byref(z))
        assert d.value == D
        assert round((z.value - d.value) / d.value, 2) == nnzr


def test_hubbard_row_lengths_and_canonical_csr():
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    rl = np.diff(A.rowptr)
    assert rl.min() == 5 and rl.max() == 17
    for i in range(A.D):
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]].astype(np.int64)
        assert np.all(np.diff(c) > 0)
        assert i in c


def test_hubbard_bitwise_symmetric():
    for L, N, U in [(6, 3, 4.0), (8, 4, 4.0), (7, 2, 2.5)]:
        Ad = O.hubbard(L, N, N, 1.0, U).dense()
        assert np.array_equal(Ad, Ad.T)


def _free_fermion_spectrum(L, nup, ndn, t):
    eps = -2.0 * t * np.cos(2 * np.pi * np.arange(L) / L)
    up = [sum(eps[list(s)]) for s in itertools.combinations(range(L), nup)]
    dn = [sum(eps[list(s)]) for s in itertools.combinations(range(L), ndn)]
    return np.sort(np.add.outer(up, dn).ravel())


@pytest.mark.parametrize("L,N", [(6, 2), (6, 3), (7, 3), (8, 4)])
def test_hubbard_U0_closed_form(L, N):
    """U = 0: eigenvalues are sums of -2t cos(2 pi m / L) over occupied momenta.
    Even N checks the fermion sign on the wrap bond (dropping it would shift
    the momenta to 2 pi (m + 1/2) / L)."""
    A = O.hubbard(L, N, N, 1.0, 0.0)
    ev = np.linalg.eigvalsh(A.dense())
    np.testing.assert_allclose(ev, _free_fermion_spectrum(L, N, N, 1.0), atol=1e-12)


def test_hubbard_particle_hole_mirror_and_zero_level():
    """Half filling, even L: spectrum symmetric about U L / 4; E = 0 exact
    (S_z = 0 member of the fully polarised multiplet)."""
    L, N, U = 6, 3, 4.0
    ev = np.linalg.eigvalsh(O.hubbard(L, N, N, 1.0, U).dense())
    np.testing.assert_allclose(ev + ev[::-1], U * L / 2, atol=1e-11)
    assert np.min(np.abs(ev)) < 1e-12


def test_anderson_counts_and_values():
    L = 6
    A = O.anderson(L, 1.0, 16.5, seed=1)
    assert A.D == L ** 3 and A.nnz == 7 * L ** 3
    Ad = A.dense()
    assert np.array_equal(Ad, Ad.T)
    off = Ad - np.diag(np.diag(Ad))
    assert set(np.unique(off)) == {0.0, -1.0}
    assert np.all((off != 0).sum(axis=1) == 6)
    # disorder drawn from the seeded stream in row order
    np.testing.assert_array_equal(np.diag(Ad), 16.5 * (O.uniforms(1, L ** 3) - 0.5))


def test_anderson_W0_closed_form():
    L = 9
    ev = np.linalg.eigvalsh(O.anderson(L, 1.0, 0.0).dense())
    k = 2 * np.pi * np.arange(L) / L
    c = np.cos(k)
    want = np.sort((-2.0 * (c[:, None, None] + c[None, :, None] + c[None, None, :])).ravel())
    np.testing.assert_allclose(ev, want, atol=1e-12)


def test_anderson_traces():
    L, W = 7, 10.0
    A = O.anderson(L, 1.0, W, seed=3)
    ev = np.linalg.eigvalsh(A.dense())
    eps = W * (O.uniforms(3, L ** 3) - 0.5)
    assert abs(ev.sum() - eps.sum()) < 1e-9
    assert abs((ev ** 2).sum() - ((eps ** 2).sum() + 6 * L ** 3)) < 1e-8


def test_gershgorin_encloses_spectrum():
    for A in (O.hubbard(6, 3, 3, 1.0, 4.0), O.anderson(5, 1.0, 16.5)):
        lo, hi = O.gershgorin(A)
        ev = np.linalg.eigvalsh(A.dense())
        assert lo <= ev[0] and ev[-1] <= hi
    assert O.gershgorin(O.hubbard(8, 4, 4, 1.0, 4.0)) == (-16.0, 32.0)
    assert O.gershgorin(O.hubbard(6, 3, 3, 1.0, 4.0)) == (-12.0, 24.0)


@pytest.mark.parametrize("C_,sigma", [(1, 1), (4, 1), (8, 32), (32, 128), (64, 1 << 20)])
def test_sell_definition(C_, sigma):
    """SELL-C-sigma structural definition, checked independently of the fill."""
    A = O.hubbard(7, 3, 2, 1.0, 3.0)
    S = O.sell(A, C_, sigma)
    D = A.D
    rl = np.diff(A.rowptr)
    perm = S.perm.astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(D))
    for w in range(0, D, sigma):
        seg = perm[w:w + sigma]
        # descending length, ties in original order (stable)
        keys = list(zip(-rl[seg], seg))
        assert keys == sorted(keys)
    nch = (D + C_ - 1) // C_
    for c in range(nch):
        rows = perm[c * C_:(c + 1) * C_]
        assert S.chunk_len[c] == rl[rows].max()
        assert S.chunk_ptr[c + 1] - S.chunk_ptr[c] == C_ * S.chunk_len[c]
        for r in range(C_):
            s = c * C_ + r
            for j in range(S.chunk_len[c]):
                at = S.chunk_ptr[c] + j * C_ + r
                if s >= D:
                    assert S.col[at] == 0 and S.val[at] == 0.0
                    continue
                o = perm[s]
                if j < rl[o]:
                    assert S.col[at] == A.col[A.rowptr[o] + j]
                    assert S.val[at] == A.val[A.rowptr[o] + j]
                else:
                    assert S.col[at] == o and S.val[at] == 0.0
