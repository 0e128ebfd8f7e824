"""Assembled (CSR) saddle systems for the tests: the MAC operators of a
small grid assembled by the oracle (restricted to the unknowns), and a
random system that no grid produces (a weighted graph Laplacian plus a
shift for W, a random sparse full-column-rank A).  Test infrastructure: only
the oracle's operators are applied here."""
import numpy as np
import scipy.sparse as sp

import oracle
import problems as P


def mac_system(grid, mu=None):
    """(W, A, face mask, cell mask): the oracle's W and A on the unknowns of
    the grid as scipy CSR matrices."""
    fm, cm = grid.face_mask() > 0, grid.cell_mask() > 0
    W = oracle.dense(grid, "W", mu=mu)[np.ix_(fm, fm)]
    A = oracle.dense(grid, "A")[np.ix_(fm, cm)]
    W[np.abs(W) < 1e-300] = 0.0
    A[np.abs(A) < 1e-300] = 0.0
    return sp.csr_matrix(W), sp.csr_matrix(A), fm, cm


def random_system(m, n, seed, density=0.02):
    """W = L + 0.1 I with L the Laplacian of a random weighted graph on m
    nodes (SPD, rows of different scales), A sparse m x n with a dense
    identity-like part so that it has full column rank, entries of
    different magnitudes per column (so central scaling matters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    G = sp.random(m, m, density=density, random_state=np.random.RandomState(seed),
                  data_rvs=lambda k: rng.uniform(0.1, 10.0, k))
    G = G + G.T
    L = sp.diags(np.asarray(G.sum(axis=1)).ravel()) - G
    W = (L + sp.diags(rng.uniform(0.1, 1.0, m))).tocsr()
    A = sp.random(m, n, density=density, random_state=np.random.RandomState(seed + 1),
                  data_rvs=lambda k: rng.standard_normal(k)).tolil()
    for k in range(n):  # a guaranteed pivot per column
        A[k, k] = 1.0 + rng.uniform(0.0, 1.0)
    A = (A.tocsr() @ sp.diags(10.0 ** rng.uniform(-2, 2, n))).tocsr()
    return W, A


def dense_solution(W, A, g, r):
    """Exact solution of [[W, A], [A^T, 0]] [w; p] = [g; r] by LU."""
    Wd, Ad = W.toarray(), A.toarray()
    K = np.block([[Wd, Ad], [Ad.T, np.zeros((Ad.shape[1],) * 2)]])
    x = np.linalg.solve(K, np.concatenate([g, r]))
    return x[:W.shape[0]], x[W.shape[0]:]


def rhs(m, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(m), rng.standard_normal(n)


__all__ = ["mac_system", "random_system", "dense_solution", "rhs", "P"]
