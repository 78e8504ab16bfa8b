"""Lehmann intervals on the GPU (fd_lehmann, and the Lehmann-controlled
filter window of fd_solve, adapt = 2) against the oracle and the dense
spectrum.

The pencil eigenvalues mu are computed from three Gram products, a Cholesky
factor and a symmetric eigensolve; the bounds are rho + 1/mu.  Parity: the
same number of bounds on each side, and distances |bound - rho| within 1e-9
relative of the oracle's (bounds farther than 10 ||H|| from rho are
uninformative and not compared).  The inclusion theorem is checked on the
GPU's own bounds against the dense spectrum.
"""
import numpy as np
import pytest

import oracle as O
from fd_inputs import start_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2209_01974_amd as fd  # noqa: E402


def subspace(A, k, rho, seed, degree=12):
    alpha, beta = O.scaling(*O.gershgorin(A))
    V = O.cheb_filter(A, start_block(A.D, k, seed), O.cheb_coeffs(1, alpha * rho + beta, 0.0, degree), alpha,
                      beta)
    V, _ = O.svqb2(V)
    return V


@pytest.mark.parametrize("name,k,rho", [("and8", 40, 0.3), ("and8", 64, -2.0), ("hub6", 33, 2.01),
                                        ("hub6", 128, 0.37), ("and8", 5, 0.0)])
def test_lehmann_parity_and_inclusion(name, k, rho):
    A = O.anderson(8, 1.0, 8.0, 4) if name == "and8" else O.hubbard(6, 3, 3, 1.0, 4.0)
    normH = max(abs(x) for x in O.gershgorin(A))
    lam = np.linalg.eigvalsh(A.dense())
    V = subspace(A, k, rho, 8)
    W = O.spmmv(A, V)
    lo, up = fd.lehmann(torch.from_numpy(V).cuda(), torch.from_numpy(W).cuda(), rho)
    lo_o, up_o, _ = O.lehmann(A, V, rho)
    assert (lo.size, up.size) == (lo_o.size, up_o.size)
    for g, o in ((rho - lo, rho - lo_o), (up - rho, up_o - rho)):
        near = o <= 10 * normH
        assert np.all(np.abs(g[near] - o[near]) <= 1e-9 * o[near])
    for i, b in enumerate(lo):
        assert np.sum((lam >= b) & (lam < rho)) >= i + 1
    for i, b in enumerate(up):
        assert np.sum((lam > rho) & (lam <= b)) >= i + 1


def test_lehmann_exact_eigenvectors_and_errors():
    A = O.anderson(6, 1.0, 8.0, 4)
    lam, X = np.linalg.eigh(A.dense())
    idx = [3, 50, 100, 101, 180]
    V = np.ascontiguousarray(X[:, idx])
    W = O.spmmv(A, V)
    rho = 0.5 * (lam[100] + lam[101])
    lo, up = fd.lehmann(torch.from_numpy(V).cuda(), torch.from_numpy(W).cuda(), rho)
    np.testing.assert_allclose(lo, np.sort(lam[idx][lam[idx] < rho])[::-1], atol=1e-10 * 12)
    np.testing.assert_allclose(up, np.sort(lam[idx][lam[idx] > rho]), atol=1e-10 * 12)
    Vd = torch.from_numpy(V).cuda()
    with pytest.raises(fd.FDError) as e:  # rho not finite
        fd.lehmann(Vd, torch.from_numpy(W).cuda(), float("nan"))
    assert e.value.status == fd.FD_ERR_INVALID
    with pytest.raises(fd.FDError):  # V and W the same block
        fd.lehmann(Vd, Vd, 0.0)


def test_solve_lehmann_window_hubbard8_vs_dense_and_oracle():
    """adapt = 2: the filter window is tau +- the Lehmann radius.  Same
    answer as dense diagonalization and as the oracle's FD with the same
    rule and start block."""
    A = O.hubbard(8, 4, 4, 1.0, 4.0)
    ev = np.linalg.eigvalsh(A.dense())
    inside = ev[(ev >= -0.5) & (ev <= 0.5)]
    want = np.sort(inside[np.argsort(np.abs(inside), kind="stable")[:16]])
    V0 = start_block(A.D, 128, 0)
    m = fd.build_matrix("hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0)
    r = fd.solve(m, -0.5, 0.5, 16, 128, 16, 100, max_iter=80, tol=1e-9, V0=V0, adapt=2)
    assert r.status == fd.FD_OK, r.stats
    normH = r.stats["norm_H"]
    assert np.abs(r.evals - want).max() <= 1e-10 * normH
    X = r.evecs.cpu().numpy()
    assert np.linalg.norm(O.spmmv(A, X) - X * r.evals, axis=0).max() <= 1e-9 * normH
    ro = O.fd_solve(A, V0, -0.5, 0.5, 16, 100, 1e-9, max_iter=80, adapt=2)
    assert ro.converged and abs(ro.iters - r.stats["iters"]) <= 1
    assert np.abs(ro.evals - r.evals).max() <= 1e-10 * normH
