"""The assembled-matrix (CSR) front end with central block scaling (paper
Section 3: the user passes the blocks; Section 4.1: the scaling by
blockdiag(D^-1/2, R^-1/2)) through the C-ABI, against the oracle's CSR path
on the same matrices and right-hand sides: element by element at equal K,
with and without scaling, in FP64, plus the mixed-precision and FGMRES
variants by the oracle's residual, and the argument checks."""
import numpy as np
import pytest

import oracle
import problems as P
from csr_cases import dense_solution, mac_system, random_system, rhs

D, N = P.DIRICHLET, P.NATURAL
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(x):
    import torch
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _systems():
    out = []
    g2 = P.Grid(2, (24, 16, 1), 1 / 24, (D,) * 6, 0)
    W, A, _, _ = mac_system(g2)
    out.append(("mac2d_24x16_eta10", W, A, 10.0))
    g3 = P.Grid(3, (8, 6, 6), 1 / 8, (D, N, D, D, D, D), -1)
    mu = np.exp(np.random.default_rng(2).standard_normal(g3.n_cells))
    W, A, _, _ = mac_system(g3, mu)
    out.append(("mac3d_outflow_varmu_eta1", W, A, 1.0))
    W, A = random_system(900, 200, 5)
    out.append(("random_900x200_eta1", W, A, 1.0))
    return out


SYSTEMS = _systems()


@pytest.mark.parametrize("scaling", ["none", "central"])
@pytest.mark.parametrize("si", range(len(SYSTEMS)), ids=[s[0] for s in SYSTEMS])
def test_csr_gkb_parity(si, scaling):
    """Jacobi-PCG inner solves at 1e-13: a fixed number of steps, equal to
    the oracle's CSR path to relative 1e-10, and a run to the stopping rule
    with the oracle's K and result; the scaled run returns the solution of the
    given system.  The unscaled random system (column scales over four
    decades) needs about 1300 GKB steps, far past the loss of orthogonality,
    where rounding moves the step at which the bound crosses tau (the oracle
    itself stops at 1282 or 1285 steps with 8 or 16 threads): there the
    criterion run is compared by K within 1 % and by its distance to the LU
    solution; with central scaling the same system takes 23 steps."""
    name, W, A, eta = SYSTEMS[si]
    _say("csr parity", name, scaling)
    import paper_2001_10424_amd as gk
    m, n = A.shape
    g, r = rhs(m, n, 8)
    for tol, maxit in ((0.0, 6), (1e-9, 2000)):
        s = gk.CsrSolver(W, A, eta, scaling=scaling, inner_tol=1e-13, inner_maxit=200000,
                         maxit=maxit)
        assert (s.m_full, s.n_cells, s.m_unknown, s.n_unknown) == (m, n, m, n)
        w, p, info = s.solve(_dev(g), _dev(r), tol=tol, delay=5)
        s.close()
        ref = oracle.gkb_solve_csr(W, A, g, r, eta, scaling=(scaling == "central"), tol=tol,
                                   delay=5, maxit=maxit, inner_tol=1e-13, inner_maxit=200000)
        assert info["status"] == ref["status"] == (0 if tol > 0 else 1)
        w, p = w.cpu().numpy(), p.cpu().numpy()
        if ref["K"] > 500:
            assert abs(info["iterations"] - ref["K"]) <= 0.01 * ref["K"], (info["iterations"],
                                                                          ref["K"])
            continue
        assert info["iterations"] == ref["K"]
        assert _rel(w, ref["w"]) <= 1e-10 and _rel(p, ref["p"]) <= 1e-10, (_rel(w, ref["w"]),
                                                                             _rel(p, ref["p"]))
    ws, ps = dense_solution(W, A, g, r)
    assert _rel(w, ws) <= 1e-6 and _rel(p, ps) <= 1e-6
    if name.startswith("random"):
        print("GKB steps to tau = 1e-9:", info["iterations"], "scaling", scaling, flush=True)


def test_csr_operators_and_residual():
    """gkb_apply on a CSR context applies the (scaled) operators of the
    iteration: with central scaling diag(W') = 1 and A'^T A' has a unit
    diagonal; gkb_residual evaluates the given system, element by element
    against the dense blocks."""
    _say("csr operators")
    import torch

    import paper_2001_10424_amd as gk
    W, A = random_system(700, 150, 9)
    m, n = A.shape
    sw, sp = oracle.csr_central_scaling(W, A)
    s = gk.CsrSolver(W, A, 0.0, scaling="central")
    d = s.apply("diag", None).cpu().numpy()
    np.testing.assert_allclose(d, 1.0, rtol=1e-14)
    x = np.random.default_rng(1).standard_normal(m)
    pc = np.random.default_rng(2).standard_normal(n)
    Wd, Ad = W.toarray(), A.toarray()
    Ws = sw[:, None] * Wd * sw[None, :]
    As = sw[:, None] * Ad * sp[None, :]
    for op, ref, xin in (("W", Ws @ x, x), ("A", As @ pc, pc), ("AT", As.T @ x, x)):
        y = s.apply(op, _dev(xin)).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), op
    g, r = rhs(m, n, 3)
    w, p = np.random.default_rng(4).standard_normal(m), np.random.default_rng(5).standard_normal(n)
    norms, rw, rr = s.residual(_dev(g), _dev(r), _dev(w), _dev(p), want_vectors=True)
    rw_ref, rr_ref = g - Wd @ w - Ad @ p, r - Ad.T @ w
    assert np.abs(rw.cpu().numpy() - rw_ref).max() <= 1e-12 * np.abs(rw_ref).max()
    assert np.abs(rr.cpu().numpy() - rr_ref).max() <= 1e-12 * np.abs(rr_ref).max()
    total = np.sqrt(np.sum(rw_ref ** 2) + np.sum(rr_ref ** 2))
    assert abs(norms[0] - total) <= 1e-12 * total
    s.close()
    del torch


@pytest.mark.parametrize("precision,krylov", [("mixed", "cg"), ("fp64", "fgmres"),
                                              ("mixed", "fgmres")])
def test_csr_mixed_and_fgmres(precision, krylov):
    """FP32 inner solves with FP64 defect correction, and FGMRES inner
    solves, on the random system with central scaling: the oracle's FP64
    residual of the given system meets 1e-8."""
    _say("csr", precision, krylov)
    import paper_2001_10424_amd as gk
    W, A = random_system(900, 200, 5)
    m, n = A.shape
    g, r = rhs(m, n, 6)
    s = gk.CsrSolver(W, A, 1.0, scaling="central", precision=precision, krylov=krylov,
                     inner_tol=1e-5 if precision == "mixed" else 1e-11, inner_maxit=50000,
                     maxit=2000, refine_tol=1e-11, max_sweeps=40)
    w, p, info = s.solve(_dev(g), _dev(r), tol=1e-3 if precision == "mixed" else 1e-10, delay=3)
    w, p = w.cpu().numpy(), p.cpu().numpy()
    Wd, Ad = W.toarray(), A.toarray()
    res = np.concatenate([g - Wd @ w - Ad @ p, r - Ad.T @ w])
    rel = np.linalg.norm(res) / np.linalg.norm(np.concatenate([g, r]))
    print("sweeps", info["sweeps"], "K", info["outer_iterations"], "inner",
          info["inner_iterations"], "residual", rel, flush=True)
    assert rel <= 1e-8
    norms, _, _ = s.residual(_dev(g), _dev(r), _dev(w), _dev(p))
    # both residuals are formed in FP64 in different orders: they agree to the
    # rounding bound of forming b - Kx, a few eps times |K||x| + |b|
    Wa, Aa = np.abs(Wd), np.abs(Ad)
    scale = np.linalg.norm(np.concatenate([Wa @ np.abs(w) + Aa @ np.abs(p) + np.abs(g),
                                           Aa.T @ np.abs(w) + np.abs(r)]))
    bnorm = np.linalg.norm(np.concatenate([g, r]))
    assert abs(norms[0] / norms[3] - rel) <= 1e-6 * rel + 64 * 2.0 ** -52 * scale / bnorm
    s.close()


def test_csr_argument_checks():
    _say("csr errors")
    import scipy.sparse as sp

    import paper_2001_10424_amd as gk
    W, A = random_system(60, 12, 2)
    with pytest.raises(RuntimeError, match="gkb_setup_csr"):
        gk.CsrSolver(W, A, 1.0, inner="mg")  # multigrid needs a grid
    with pytest.raises(RuntimeError, match="gkb_setup_csr"):
        gk.CsrSolver(W, A, -1.0)
    Wz = W.tolil()
    Wz[3, 3] = 0.0
    with pytest.raises(RuntimeError, match="gkb_setup_csr"):
        gk.CsrSolver(Wz.tocsr(), A, 1.0)  # non-positive diagonal of W
    A0 = A.tolil()
    A0[:, 5] = 0.0
    A0 = sp.csr_matrix(A0.toarray())
    with pytest.raises(RuntimeError, match="gkb_setup_csr"):
        gk.CsrSolver(W, A0, 1.0, scaling="central")  # empty column of A
    s = gk.CsrSolver(W, A0, 1.0, scaling="none")  # allowed unscaled (eta > 0 keeps M definite)
    s.close()
