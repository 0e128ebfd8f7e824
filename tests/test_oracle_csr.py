"""Pins of the oracle's assembled-matrix (CSR) path and of the central
scaling of Section 4.1: the same GKB as the matrix-free MAC operators on the
same matrices, invariants of the scaling, and exact solutions by LU."""
import numpy as np
import pytest

import oracle
import problems as P
from csr_cases import dense_solution, mac_system, random_system, rhs

D, N = P.DIRICHLET, P.NATURAL

GRIDS = [
    (P.Grid(2, (8, 6, 1), 1 / 8, (D,) * 6, 0), 10.0, False),
    (P.Grid(2, (12, 4, 1), 0.25, (D, N, D, D, D, D), -1), 1e2, True),
    (P.Grid(3, (4, 4, 3), 0.25, (D,) * 6, 0), 0.0, True),
]


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_csr_path_equals_mac_path(gi):
    """Unscaled, the CSR path runs the same GKB as the MAC operators on the
    assembled matrices: same K, results equal up to the amplification of
    rounding by kappa(M) * tau_in (the products sum in a different order;
    relative 1e-10, the parity bound of the GPU path)."""
    grid, eta, varmu = GRIDS[gi]
    mu = np.exp(np.random.default_rng(5).standard_normal(grid.n_cells)) if varmu else None
    W, A, fm, cm = mac_system(grid, mu)
    gv = P.random_vector(grid, 1)
    rv = P.random_vector(grid, 2, "cells")
    for tol, maxit in ((0.0, 5), (1e-9, 400)):
        ref = oracle.gkb_solve(grid, gv, rv, eta, mu=mu, tol=tol, delay=3, maxit=maxit,
                               inner_tol=1e-13)
        res = oracle.gkb_solve_csr(W, A, gv[fm], rv[cm], eta, scaling=False, tol=tol, delay=3,
                                   maxit=maxit, inner_tol=1e-13)
        assert res["status"] == ref["status"] and res["K"] == ref["K"]
        for a, b in ((res["w"], ref["w"][fm]), (res["p"], ref["p"][cm])):
            assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("case", ["mac", "random"])
def test_central_scaling_invariants(case):
    """s_w = diag(W)^-1/2 and s_p = diag(A^T D^-1 A)^-1/2 equilibrate the
    blocks: the scaled W has unit diagonal and the columns of the scaled A
    have unit 2-norm."""
    if case == "mac":
        W, A, _, _ = mac_system(GRIDS[1][0], np.exp(np.random.default_rng(5).standard_normal(48)))
    else:
        W, A = random_system(300, 80, 3)
    sw, sp_ = oracle.csr_central_scaling(W, A)
    Ws = W.multiply(np.outer(sw, sw)).toarray()
    As = (A.toarray() * sw[:, None]) * sp_[None, :]
    np.testing.assert_allclose(np.diag(Ws), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.sum(As * As, axis=0), 1.0, rtol=1e-13)
    with pytest.raises(ValueError):  # an empty column of A
        A0 = A.tolil()
        A0[:, 0] = 0.0
        oracle.csr_central_scaling(W, A0.tocsr())


@pytest.mark.parametrize("scaling", [False, True])
@pytest.mark.parametrize("case", ["mac", "random"])
def test_csr_gkb_matches_dense_lu(case, scaling):
    """Run past the exhaustion of the Krylov space: the exact solution of the
    given (unscaled) system, with or without central scaling."""
    if case == "mac":
        grid, eta, _ = GRIDS[0]
        W, A, _, _ = mac_system(grid)
    else:
        W, A = random_system(240, 50, 7)
        eta = 1.0
    m, n = A.shape
    g, r = rhs(m, n, 3)
    ws, ps = dense_solution(W, A, g, r)
    res = oracle.gkb_solve_csr(W, A, g, r, eta, scaling=scaling, tol=0.0, maxit=3 * n,
                               inner_tol=1e-14)
    assert np.linalg.norm(res["w"] - ws) <= 1e-10 * np.linalg.norm(ws)
    assert np.linalg.norm(res["p"] - ps) <= 1e-10 * np.linalg.norm(ps)


def test_scaling_changes_iterates_not_solution():
    """On the random system (column scales 1e-2 ... 1e2) the scaled GKB needs
    fewer steps to the same lower-bound tolerance and both meet the exact
    solution to the accuracy that tolerance implies."""
    W, A = random_system(400, 90, 11)
    m, n = A.shape
    g, r = rhs(m, n, 4)
    ws, ps = dense_solution(W, A, g, r)
    out = {}
    for scaling in (False, True):
        res = oracle.gkb_solve_csr(W, A, g, r, 1.0, scaling=scaling, tol=1e-10, delay=5,
                                   maxit=2000, inner_tol=1e-13)
        assert res["status"] == 0
        assert np.linalg.norm(res["w"] - ws) <= 1e-6 * np.linalg.norm(ws)
        out[scaling] = res["K"]
    assert out[True] < out[False], out
