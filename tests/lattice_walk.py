"""Tiled site numbering of the 3D lattice, written out for the tests: the
walk over (x, y) tiles and the symmetric permutation B = P A P^T it gives."""
import numpy as np

import oracle as O


def tile_walk(L, tx, ty):
    """Sites of the L^3 lattice (natural index x + L y + L^2 z) in (x, y)
    tiles of tx by ty, tiles in x-then-y order, each tile over all z (z
    outermost, then y, then x)."""
    parts = []
    for y0 in range(0, L, ty):
        for x0 in range(0, L, tx):
            z, y, x = np.meshgrid(np.arange(L), np.arange(y0, min(L, y0 + ty)), np.arange(x0, min(L, x0 + tx)),
                                  indexing="ij")
            parts.append((x + L * y + L * L * z).ravel())
    return np.concatenate(parts).astype(np.int64)


def permuted_csr(A, p):
    """B = P A P^T: row r of B is row p[r] of A, columns renamed by the
    inverse of p and sorted."""
    inv = np.empty_like(p)
    inv[p] = np.arange(p.size)
    rowptr, cols, vals = [0], [], []
    for o in p:
        a, b = A.rowptr[o], A.rowptr[o + 1]
        c = inv[A.col[a:b].astype(np.int64)]
        order = np.argsort(c, kind="stable")
        cols.append(c[order])
        vals.append(A.val[a:b][order])
        rowptr.append(rowptr[-1] + (b - a))
    return O.CSR(A.D, np.array(rowptr, np.int64), np.concatenate(cols).astype(np.uint32), np.concatenate(vals))


def anderson_tiled(L, t, W, seed, tx, ty):
    """The oracle's Anderson matrix with its sites numbered along the walk."""
    return permuted_csr(O.anderson(L, t, W, seed), tile_walk(L, tx, ty))
