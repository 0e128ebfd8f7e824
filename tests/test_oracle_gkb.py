"""Pins of the oracle's GKB solver (paper Section 2, Algorithm 1, stopping rule
of Section 2.2) and of its Jacobi-PCG inner solve against dense linear
algebra and the algebraic identities of the method."""
import numpy as np
import pytest

import oracle
import problems as P

D, N = P.DIRICHLET, P.NATURAL

CASES = [
    # (grid, eta, variable viscosity)
    (P.Grid(2, (8, 2, 1), 0.5, (D, N, D, D, D, D), -1), 100.0, False),
    (P.Grid(2, (16, 4, 1), 0.25, (D, N, D, D, D, D), -1), 100.0, False),
    (P.Grid(2, (4, 4, 1), 0.25, (D,) * 6, 0), 0.0, False),
    (P.Grid(2, (8, 8, 1), 0.125, (D,) * 6, 0), 10.0, True),
    (P.Grid(3, (4, 4, 4), 0.25, (D,) * 6, 0), 10.0, False),
    (P.Grid(3, (4, 4, 4), 0.25, (D,) * 6, 0), 0.0, True),
]


def _mu(g, on):
    return np.exp(np.random.default_rng(11).standard_normal(g.n_cells)) if on else None


def _dense(g, eta, mu):
    fm, cm = g.face_mask() > 0, g.cell_mask() > 0
    W = oracle.dense(g, "W", mu=mu)[np.ix_(fm, fm)]
    A = oracle.dense(g, "A")[np.ix_(fm, cm)]
    M = W + eta * A @ A.T
    return fm, cm, W, A, M


@pytest.mark.parametrize("krylov", ["cg", "fgmres"])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_gkb_matches_dense_lu(ci, krylov):
    """Run to breakdown / K = n: the result is the exact solution of the
    saddle-point system, as given by LU (numpy.linalg.solve), with either
    inner Krylov method (FGMRES restarted every 7 steps, so the restart path
    runs).  Restarted FGMRES with point Jacobi stagnates just above 1e-14 on
    the channels (its true residual, which decides the stop, stays there), so
    it runs at inner tolerance 1e-13, whose errors of order kappa(M) * 1e-13
    per inner solve (kappa(M) = 585 on the 16 x 4 channel) accumulate over
    the 3n steps: bound 5e-11 against 1e-12 for CG at 1e-14."""
    g, eta, varmu = CASES[ci]
    tol = 1e-12 if krylov == "cg" else 5e-11
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    gv = P.random_vector(g, 1)
    rv = P.random_vector(g, 2, "cells")
    K = np.block([[W, A], [A.T, np.zeros((A.shape[1],) * 2)]])
    sol = np.linalg.solve(K, np.concatenate([gv[fm], rv[cm]]))
    res = oracle.gkb_solve(g, gv, rv, eta, mu=mu, tol=0.0, maxit=3 * cm.sum(),
                           inner_tol=1e-14 if krylov == "cg" else 1e-13, krylov=krylov,
                           restart=7)
    w, p = res["w"][fm], res["p"][cm]
    ws, ps = sol[:fm.sum()], sol[fm.sum():]
    assert np.linalg.norm(w - ws) <= tol * np.linalg.norm(ws)
    assert np.linalg.norm(p - ps) <= tol * np.linalg.norm(ps)
    # non-unknown entries are written as zero
    assert np.all(res["w"][~fm] == 0) and np.all(res["p"][~cm] == 0)


@pytest.mark.parametrize("ci", [0, 2, 4, 5])
def test_bidiagonal_singular_values(ci):
    """B of the generalized bidiagonalization carries the singular values of
    M^{-1/2} A N^{-1/2} (Section 2.1): the extreme ones after n steps, and
    after 3n steps every one (finite-precision GKB repeats converged values
    instead of losing them)."""
    g, eta, varmu = CASES[ci]
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    n = cm.sum()
    L = np.linalg.cholesky(M)
    sv = np.linalg.svd(np.linalg.solve(L, A) * (np.sqrt(eta) if eta > 0 else 1.0),
                       compute_uv=False)
    gv = P.random_vector(g, 1)
    rv = P.random_vector(g, 2, "cells")
    res = oracle.gkb_solve(g, gv, rv, eta, mu=mu, tol=0.0, maxit=3 * n, inner_tol=1e-14)
    K = res["K"]
    assert K == 3 * n
    for k in (n, K):
        B = np.diag(res["alpha"][:k]) + np.diag(res["beta"][1:k], 1)
        sb = np.linalg.svd(B, compute_uv=False)
        assert abs(sb.max() - sv.max()) <= 1e-12 * sv.max()
        assert abs(sb.min() - sv.min()) <= 1e-10 * sv.min()
        # interlacing: no value outside [sigma_min, sigma_max]
        assert sb.min() >= sv.min() * (1 - 1e-10) and sb.max() <= sv.max() * (1 + 1e-12)
    B = np.diag(res["alpha"][:K]) + np.diag(res["beta"][1:K], 1)
    sb = np.linalg.svd(B, compute_uv=False)
    dist = max(np.abs(sb - s).min() for s in sv)
    assert dist <= 1e-10 * sv.max()


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_generalized_gk_relations(ci):
    """A Q = M V B and A^T V = N Q B^T + beta_{k+1} N q_{k+1} e_k^T, with
    V^T M V = I and Q^T N Q = I on the first columns (Section 2.1)."""
    g, eta, varmu = CASES[ci]
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    n = cm.sum()
    k = min(n, 12)
    gv = P.random_vector(g, 1)
    rv = P.random_vector(g, 2, "cells")
    res = oracle.gkb_solve(g, gv, rv, eta, mu=mu, tol=0.0, maxit=k + 1,
                           inner_tol=1e-14, store_k=k + 1)
    V = res["V"][:, fm].T
    Q = res["Q"][:, cm].T
    Nm = (1.0 / eta) if eta > 0 else 1.0
    B = np.diag(res["alpha"][:k]) + np.diag(res["beta"][1:k], 1)
    scale = np.abs(A).max()
    assert np.abs(A @ Q[:, :k] - M @ V[:, :k] @ B).max() <= 1e-11 * scale * np.abs(V).max() * 10
    E = np.zeros((k, k))
    rhs = Nm * Q[:, :k] @ B.T
    rhs[:, k - 1] += res["beta"][k] * Nm * Q[:, k]
    assert np.abs(A.T @ V[:, :k] - rhs).max() <= 1e-10 * np.abs(A.T @ V[:, :k]).max()
    j = 4
    assert np.abs(V[:, :j].T @ M @ V[:, :j] - np.eye(j)).max() <= 1e-10
    assert np.abs(Nm * Q[:, :j].T @ Q[:, :j] - np.eye(j)).max() <= 1e-10
    del E


@pytest.mark.parametrize("ci", [1, 3, 4])
def test_zeta_energy_identity_and_lower_bound(ci):
    """With g chosen so that the transformed first right-hand side vanishes
    (g = -gamma A N^-1 r, hence w0 = 0 and u = w):
      sum_{j<=k} zeta_j^2 = ||u_k||_M^2 (non-decreasing, -> ||u||_M^2),
      ||u - u_k||_M^2 = sum_{j>k} zeta_j^2, and the delayed lower bound
      xi_{k,d}^2 = sum_{j=k+1}^{k+d+1} zeta_j^2 <= ||e_k||_M^2 (Section 2.2)."""
    g, eta, varmu = CASES[ci]
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    rv = P.random_vector(g, 2, "cells")
    gv = -eta * oracle.apply_A(g, rv * g.cell_mask())
    n = cm.sum()
    full = oracle.gkb_solve(g, gv, rv, eta, mu=mu, tol=0.0, maxit=3 * n, inner_tol=1e-14)
    Kz = np.cumsum(full["zeta"] ** 2)
    Kd = np.block([[W, A], [A.T, np.zeros((n, n))]])
    u = np.linalg.solve(Kd, np.concatenate([gv[fm], rv[cm]]))[:fm.sum()]
    uMu = u @ M @ u
    assert np.all(np.diff(Kz) >= -1e-14 * uMu)
    assert abs(Kz[n - 1] - uMu) <= 1e-9 * uMu
    d = 3
    for k in range(1, min(n - d - 1, 10)):
        part = oracle.gkb_solve(g, gv, rv, eta, mu=mu, tol=0.0, maxit=k, inner_tol=1e-14)
        uk = part["w"][fm]
        assert abs(uk @ M @ uk - Kz[k - 1]) <= 1e-10 * uMu
        e = u - uk
        eM2 = e @ M @ e
        assert abs(eM2 - (uMu - Kz[k - 1])) <= 1e-9 * uMu
        xi2 = np.sum(full["zeta"][k:k + d + 1] ** 2)
        assert xi2 <= eM2 + 1e-13 * uMu


def test_stopping_rule_and_delay():
    """The solve stops at the first K >= d+1 whose lower-bound ratio
    sqrt(sum_{j=K-d}^K zeta_j^2 / sum_{j<=K} zeta_j^2) is <= tau."""
    pr = P.poiseuille_problem(32, 8, 4.0, 1e2)
    g = pr.grid
    for tol, d in [(1e-4, 5), (1e-8, 5), (1e-6, 2), (1e-6, 0)]:
        res = oracle.gkb_solve(g, pr.g, pr.r, pr.eta, tol=tol, delay=d, maxit=400,
                               inner_tol=1e-13)
        K, z = res["K"], res["zeta"]
        assert res["status"] == 0
        ratios = [np.sqrt(np.sum(z[k - d - 1:k] ** 2) / np.sum(z[:k] ** 2))
                  for k in range(d + 1, K + 1)]
        assert ratios[-1] <= tol and all(r > tol for r in ratios[:-1])
        assert abs(res["est"] - ratios[-1]) <= 1e-15
        # the literal squared comparison stops earlier (tau applies to squares)
        sq = oracle.gkb_solve(g, pr.g, pr.r, pr.eta, tol=tol, delay=d, maxit=400,
                              inner_tol=1e-13, squared_rule=True)
        assert sq["K"] <= K


def test_maxit_returns_last_iterate():
    pr = P.poiseuille_problem(32, 8, 4.0, 1e2)
    res = oracle.gkb_solve(pr.grid, pr.g, pr.r, pr.eta, tol=1e-12, delay=5, maxit=4,
                           inner_tol=1e-13)
    assert res["status"] == oracle.MAXIT and res["K"] == 4


def test_zero_rhs_trivial_solution():
    g = CASES[3][0]
    res = oracle.gkb_solve(g, np.zeros(g.m_full), np.zeros(g.n_cells), 10.0, tol=1e-8)
    assert res["status"] == 0 and res["K"] == 0
    assert np.all(res["w"] == 0) and np.all(res["p"] == 0)


def test_manufactured_solution_3d():
    """Discrete manufactured solution: g = W w* + A p*, r = A^T w* gives back
    (w*, p*) to the requested accuracy."""
    g = P.Grid(3, (8, 8, 8), 1 / 8, (D,) * 6, 0)
    mu = np.exp(np.random.default_rng(2).standard_normal(g.n_cells))
    ws, ps = P.random_solution(g, 5)
    gv = oracle.apply_W(g, ws, mu) + oracle.apply_A(g, ps)
    rv = oracle.apply_AT(g, ws)
    res = oracle.gkb_solve(g, gv, rv, 10.0, mu=mu, tol=1e-10, delay=5, maxit=500,
                           inner_tol=1e-13)
    assert res["status"] == 0
    assert np.linalg.norm(res["w"] - ws) <= 1e-8 * np.linalg.norm(ws)
    assert np.linalg.norm(res["p"] - ps) <= 1e-8 * np.linalg.norm(ps)


@pytest.mark.parametrize("ci", [0, 3, 5])
def test_jacobi_pcg_against_solve(ci):
    g, eta, varmu = CASES[ci]
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    f = P.random_vector(g, 7)
    x, st, it = oracle.pcg(g, f, eta, mu, tol=1e-13)
    xs = np.linalg.solve(M, f[fm])
    assert st == 0 and it > 0
    assert np.linalg.norm(x[fm] - xs) <= 1e-11 * np.linalg.norm(xs)
    # CG minimises the M-norm of the error: non-increasing over iterations
    errs = []
    for k in range(1, 12):
        xk, _, _ = oracle.pcg(g, f, eta, mu, tol=0.0, maxit=k)
        e = xk[fm] - xs
        errs.append(e @ M @ e)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs[:-1], errs[1:]))


def test_pcg_status_on_maxit():
    g, eta, _ = CASES[3]
    f = P.random_vector(g, 7)
    _, st, it = oracle.pcg(g, f, eta, None, tol=1e-14, maxit=3)
    assert st == oracle.EINNER and it == 3


def test_saddle_residual_of_exact_solution():
    g = P.Grid(2, (12, 10, 1), 0.1, (D,) * 6, 0)
    ws, ps = P.random_solution(g, 3)
    gv = oracle.apply_W(g, ws) + oracle.apply_A(g, ps)
    rv = oracle.apply_AT(g, ws)
    _, _, nr = oracle.saddle_residual(g, gv, rv, ws, ps)
    assert nr[0] <= 1e-13 * nr[3]
    _, _, nr2 = oracle.saddle_residual(g, gv, rv, ws * 0, ps * 0)
    assert abs(nr2[0] - nr2[3]) <= 1e-12 * nr2[3]


@pytest.mark.parametrize("ci", [1, 3, 4])
def test_gkb_preconditioned_fgmres(ci):
    """GKB as the right preconditioner of flexible GMRES on the whole saddle
    system (Section 3).  An exact GKB run (no stopping tolerance, run past
    the exhaustion of the Krylov space) is the exact inverse, so FGMRES stops
    after one step with the LU solution; a loose GKB run (lower-bound
    tolerance 0.3, delay 1) needs several outer steps, every one lowers the
    residual, and the result meets the requested relative residual."""
    g, eta, varmu = CASES[ci]
    mu = _mu(g, varmu)
    fm, cm, W, A, M = _dense(g, eta, mu)
    gv = P.random_vector(g, 1)
    rv = P.random_vector(g, 2, "cells")
    K = np.block([[W, A], [A.T, np.zeros((A.shape[1],) * 2)]])
    b = np.concatenate([gv[fm], rv[cm]])
    sol = np.linalg.solve(K, b)
    n = int(cm.sum())
    ex = oracle.gkb_fgmres(g, gv, rv, eta, mu=mu, tol=1e-10, restart=5, maxit=10, gkb_tol=0.0,
                           delay=1, gkb_maxit=3 * n, inner_tol=1e-14)
    assert ex["status"] == 0 and ex["iterations"] == 1
    x = np.concatenate([ex["w"][fm], ex["p"][cm]])
    assert np.linalg.norm(x - sol) <= 1e-11 * np.linalg.norm(sol)
    hist = []
    for maxit in range(1, 30):
        lo = oracle.gkb_fgmres(g, gv, rv, eta, mu=mu, tol=1e-9, restart=4, maxit=maxit,
                               gkb_tol=0.3, delay=1, gkb_maxit=3 * n, inner_tol=1e-14)
        x = np.concatenate([lo["w"][fm], lo["p"][cm]])
        hist.append(np.linalg.norm(b - K @ x))
        if lo["status"] == 0:
            break
    assert lo["status"] == 0 and lo["iterations"] >= 2
    assert hist[-1] <= 1e-9 * np.linalg.norm(b) * (1 + 1e-6)
    # FGMRES minimises the residual over a growing space within a cycle
    # (restart 4): non-increasing up to rounding
    for a, c in zip(hist[:4], hist[1:4]):
        assert c <= a * (1 + 1e-10)
    assert np.all(lo["w"][~fm] == 0) and np.all(lo["p"][~cm] == 0)
