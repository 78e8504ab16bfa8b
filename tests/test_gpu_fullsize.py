"""Full-size parity on the GPU: the measured workloads at their real sizes, in
the launch configuration the benchmark times (autotuned shape), checked on
sampled rows that the oracle computes one by one from the definition.

* 3D Anderson L=200 (D = 8,000,000, nnz = 56,000,000, W = 16.5, seed 1):
  SpMMV and degree-3 and degree-6 filters (every step form) on nb = 64, in
  the natural site numbering and in the tiled one (100 x 40 tiles), the
  latter against the natural oracle with the block permuted:
  (P A P^T X)[r] = (A P^T X)[walk[r]].
* Hubbard ring L=14, 7 up + 7 down, U=8 (D = 11,778,624, nnz = 189,364,032):
  SpMMV on nb = 32 with integer-valued blocks, bit-exact in FP64 and FP32,
  stored (CSR) and matrix-free; degree-3 and degree-4 matrix-free filters on
  nb = 32.
"""
import numpy as np
import pytest

import oracle as O
from fd_inputs import int_block, start_block
from lattice_walk import tile_walk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402

NSAMPLE = 3000


def sample_rows(D, seed):
    rng = np.random.default_rng(seed)
    r = rng.choice(D, NSAMPLE, replace=False)
    return np.sort(np.concatenate([r, [0, D - 1]]))


@pytest.fixture(scope="module")
def anderson200():
    m = fd.build_matrix("anderson", L=200, t=1.0, W=16.5, seed=1)
    A = O.anderson(200, 1.0, 16.5, 1)
    assert (m.D, m.nnz) == (8_000_000, 56_000_000)
    return m, A


def test_anderson200_spmmv_nb64_sampled(anderson200):
    m, A = anderson200
    fd.autotune(m, "f64", 64)
    X = start_block(A.D, 64, 21)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    fd.spmmv(m, Xd, Yd)
    rows = sample_rows(A.D, 1)
    got = Yd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = O.spmmv_rows(A, X, rows)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("degree,nrows", [(3, 800), (6, 200)])
def test_anderson200_filter_sampled(anderson200, degree, nrows):
    """Degree 3: the first two steps and an odd last step (V updated alone);
    degree 6: also the recurrence-only and the two-term V steps that make up
    the benchmark's filter."""
    m, A = anderson200
    fd.autotune(m, "f64", 64)
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(1, beta, 0.0, degree)
    V = start_block(A.D, 64, 22)
    Vd = torch.from_numpy(V).cuda()
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, 64)
    rows = sample_rows(A.D, 2)[:nrows]
    got = Vd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = O.cheb_filter_rows(A, V, mu, alpha, beta, rows)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12


@pytest.fixture(scope="module")
def anderson200_tiled(anderson200):
    m = fd.build_matrix("anderson", L=200, t=1.0, W=16.5, seed=1, tiles=(100, 40))
    assert (m.D, m.nnz) == (8_000_000, 56_000_000)
    walk = tile_walk(200, 100, 40)
    inv = np.empty_like(walk)
    inv[walk] = np.arange(walk.size)
    return m, anderson200[1], walk, inv


def test_anderson200_tiled_spmmv_nb64_sampled(anderson200_tiled):
    m, A, walk, inv = anderson200_tiled
    fd.autotune(m, "f64", 64)
    X = start_block(A.D, 64, 23)
    Yd = torch.empty((A.D, 64), dtype=torch.float64, device="cuda")
    fd.spmmv(m, torch.from_numpy(X).cuda(), Yd)
    rows = sample_rows(A.D, 3)
    got = Yd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = O.spmmv_rows(A, X[inv], walk[rows])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("degree,nrows", [(3, 400), (6, 150)])
def test_anderson200_tiled_filter_sampled(anderson200_tiled, degree, nrows):
    m, A, walk, inv = anderson200_tiled
    fd.autotune(m, "f64", 64)
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(1, beta, 0.0, degree)
    V = start_block(A.D, 64, 24)
    Vd = torch.from_numpy(V).cuda()
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, 64)
    rows = sample_rows(A.D, 4)[:nrows]
    got = Vd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = O.cheb_filter_rows(A, V[inv], mu, alpha, beta, walk[rows])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12


@pytest.fixture(scope="module")
def hubbard14():
    m = fd.build_matrix("hubbard", L=14, n_up=7, n_dn=7, t=1.0, U=8.0)
    A = O.hubbard(14, 7, 7, 1.0, 8.0)
    assert (m.D, m.nnz) == (11_778_624, 189_364_032)
    return m, A


@pytest.mark.parametrize("dt,bound", [(torch.float64, 1 << 10), (torch.float32, 1 << 8)])
def test_hubbard14_spmmv_nb32_integer_bit_exact(hubbard14, dt, bound):
    m, A = hubbard14
    fd.autotune(m, "f64" if dt == torch.float64 else "f32", 32)
    X = int_block(A.D, 32, 23, bound)
    Xd = torch.from_numpy(X).to(dt).cuda()
    Yd = torch.empty_like(Xd)
    fd.spmmv(m, Xd, Yd)
    rows = sample_rows(A.D, 3)
    got = Yd[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert np.array_equal(got, O.spmmv_rows(A, X, rows))


@pytest.fixture(scope="module")
def hubbard14_matfree():
    m = fd.build_matrix("hubbard", fmt="matfree", L=14, n_up=7, n_dn=7, t=1.0, U=8.0)
    assert (m.D, m.nnz) == (11_778_624, 189_364_032)
    return m


@pytest.mark.parametrize("dt,bound", [(torch.float64, 1 << 10), (torch.float32, 1 << 8)])
def test_hubbard14_matfree_spmmv_nb32_integer_bit_exact(hubbard14, hubbard14_matfree, dt, bound):
    """The matrix-free Hubbard L=14 SpMMV in its autotuned launch shape."""
    _, A = hubbard14
    m = hubbard14_matfree
    fd.autotune(m, "f64" if dt == torch.float64 else "f32", 32)
    X = int_block(A.D, 32, 24, bound)
    Xd = torch.from_numpy(X).to(dt).cuda()
    Yd = torch.empty_like(Xd)
    fd.spmmv(m, Xd, Yd)
    rows = sample_rows(A.D, 4)
    got = Yd[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert np.array_equal(got, O.spmmv_rows(A, X, rows))


@pytest.mark.parametrize("degree", [3, 4])
def test_hubbard14_matfree_filter_sampled(hubbard14, hubbard14_matfree, degree):
    """Degree-3 and degree-4 filters (first, second, recurrence-only,
    two-term and single-term V steps) on nb = 32, sampled rows against the
    oracle's neighbourhood recursion."""
    _, A = hubbard14
    m = hubbard14_matfree
    fd.autotune(m, "f64", 32)
    alpha, beta = O.scaling(*O.gershgorin(A))
    mu = O.cheb_coeffs(0, alpha * -1.0 + beta, alpha * 1.0 + beta, degree)
    V = start_block(A.D, 32, 25)
    Vd = torch.from_numpy(V).cuda()
    W1 = torch.empty_like(Vd)
    W2 = torch.empty_like(Vd)
    fd.cheb_filter(m, Vd, mu, alpha, beta, W1, W2, 32)
    rows = np.unique(np.concatenate([sample_rows(A.D, 5)[:40], [A.D - 1]]))
    got = Vd[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = O.cheb_filter_rows(A, V, mu, alpha, beta, rows)
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-12
