"""Multigrid-preconditioned inner solves and mixed precision on the GPU:
V-cycle symmetry / positivity, agreement of the LDS-tiled and generic stencil
kernels, MG-PCG against the oracle's Jacobi-PCG solution, MG-GKB parity with
the oracle at tight tolerances, and the FP64 saddle residual of mixed-precision
solves recomputed by the oracle."""
import numpy as np
import pytest

import oracle
import problems as P

D, N = P.DIRICHLET, P.NATURAL

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(x, dtype=None):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype or torch.float64, device="cuda")


def _gk():
    import paper_2001_10424_amd as gk
    return gk


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


MG_CASES = [
    ("3d32_eta1e3", P.Grid(3, (32, 32, 32), 1 / 32, (D,) * 6, 0), 1e3, False),
    ("3d_ragged_varmu", P.Grid(3, (48, 16, 24), 1 / 16, (D,) * 6, 0), 1e2, True),
    ("2d64", P.Grid(2, (64, 64, 1), 1 / 64, (D,) * 6, 0), 1e3, False),
    ("2d_channel", P.Grid(2, (64, 16, 1), 1 / 16, (D, N, D, D, D, D), -1), 1e2, False),
    ("3d_natural", P.Grid(3, (16, 16, 16), 1 / 16, (D, N, D, D, D, D), -1), 10.0, False),
]


def _mu(g, on):
    return np.exp(np.random.default_rng(5).standard_normal(g.n_cells)) if on else None


@pytest.mark.parametrize("transfer", ["div", "smooth"])
@pytest.mark.parametrize("smoother", ["jacobi", "hybrid"])
@pytest.mark.parametrize("name,grid,eta,varmu", MG_CASES, ids=[c[0] for c in MG_CASES])
def test_vcycle_symmetric_positive(name, grid, eta, varmu, smoother, transfer):
    """x.V(y) = y.V(x) and x.V(x) > 0 for both smoothers and both transfer
    pairs (restriction = prolongation^T / 2^d in each)."""
    _say("vcycle sym", name, smoother, transfer)
    gk = _gk()
    s = gk.Solver(grid, _mu(grid, varmu), eta, inner="mg", smoother=smoother,
                  mg_transfer=transfer)
    assert s.stats()["mg_transfer"] == transfer
    x = _dev(P.random_vector(grid, 1))
    y = _dev(P.random_vector(grid, 2))
    Vx = s.precondition(x)
    Vy = s.precondition(y)
    a = float((x * Vy).sum())
    b = float((y * Vx).sum())
    assert abs(a - b) <= 1e-11 * max(abs(a), abs(b)), (a, b)
    assert float((x * Vx).sum()) > 0 and float((y * Vy).sum()) > 0
    # non-unknown faces stay zero
    mask = _dev(grid.face_mask())
    assert float((Vx * (1 - mask)).abs().max()) == 0.0
    s.close()


TILED_CASES = MG_CASES[:2] + [
    ("3d_lower_natural", P.Grid(3, (16, 24, 16), 1 / 16, (N, D, D, D, D, D), -1), 10.0, True),
    ("3d_lower_natural_const", P.Grid(3, (16, 24, 16), 1 / 16, (N, D, N, D, D, D), -1), 10.0,
     False),
    ("3d_pin_mid", P.Grid(3, (16, 8, 12), 1 / 8, (D,) * 6, 5 * 16 * 8 + 3 * 16 + 7), 1e2, False),
    # two planes per tiled block, the pinned cell on the second plane of a block
    ("3d_tz2_pin", P.Grid(3, (128, 128, 32), 1 / 128, (D,) * 6, 5 * 128 * 128 + 70 * 128 + 33),
     1e2, False),
]


@pytest.mark.parametrize("smoother", ["jacobi", "hybrid"])
@pytest.mark.parametrize("name,grid,eta,varmu", TILED_CASES, ids=[c[0] for c in TILED_CASES])
def test_tiled_matches_generic(name, grid, eta, varmu, smoother):
    """The LDS-tiled 3D kernel and the generic face kernel compute the same
    operator, V-cycle (every smoother / residual mode) and inner solve."""
    _say("tiled vs generic", name, smoother)
    gk = _gk()
    mu = _mu(grid, varmu)
    s0 = gk.Solver(grid, mu, eta, inner="mg", stencil=0, smoother=smoother)
    s1 = gk.Solver(grid, mu, eta, inner="mg", stencil=1, smoother=smoother)
    x = _dev(np.random.default_rng(3).standard_normal(grid.m_full))
    for op in ("M", "W"):
        a, b = s0.apply(op, x).cpu().numpy(), s1.apply(op, x).cpu().numpy()
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    r = _dev(P.random_vector(grid, 4))
    a, b = s0.precondition(r).cpu().numpy(), s1.precondition(r).cpu().numpy()
    assert _rel(a, b) <= 1e-12
    # rounding-order differences can move the stopping iteration of a slowly
    # converging CG by a few steps; both solutions meet the tolerance
    xa, ia = s0.inner_solve(r, 1e-9)
    xb, ib = s1.inner_solve(r, 1e-9)
    assert abs(ia - ib) <= 2 + 0.03 * ib
    assert _rel(xa.cpu().numpy(), xb.cpu().numpy()) <= 1e-6
    s0.close()
    s1.close()


def test_vcycle_laplacian_convergence_factor():
    """eta = 0 (M = W, the vector Laplacian): the mean residual reduction per
    MG-PCG iteration, (1e-8)^(1 / iterations), is a textbook V(2,2) factor
    (<= 0.2) and does not grow with the grid."""
    _say("laplacian mg")
    gk = _gk()
    its = []
    for n in (16, 32, 64, 128):
        g = P.Grid(3, (n, n, n), 1 / n, (D,) * 6, 0)
        s = gk.Solver(g, None, 0.0, inner="mg")
        f = _dev(P.random_vector(g, 3))
        _, it = s.inner_solve(f, 1e-8)
        its.append(it)
        s.close()
    rho = [1e-8 ** (1.0 / k) for k in its]
    print("[case] iterations", its, "factors", [round(r, 3) for r in rho], flush=True)
    assert max(rho) <= 0.2 and its[-1] <= its[0] + 2, (its, rho)


@pytest.mark.parametrize("smoother", ["jacobi", "hybrid"])
@pytest.mark.parametrize("name,grid,eta,varmu", MG_CASES, ids=[c[0] for c in MG_CASES])
def test_mg_pcg_solution_matches_oracle(name, grid, eta, varmu, smoother):
    _say("mg-pcg vs oracle", name, smoother)
    gk = _gk()
    mu = _mu(grid, varmu)
    s = gk.Solver(grid, mu, eta, inner="mg", inner_maxit=20000, smoother=smoother)
    f = P.random_vector(grid, 6)
    x, it = s.inner_solve(_dev(f), 1e-12)
    ref, st, _ = oracle.pcg(grid, f, eta, mu, tol=1e-13, maxit=10 ** 6)
    assert st == 0
    assert _rel(x.cpu().numpy(), ref) <= 1e-7
    # residual of the GPU solution in FP64 by the oracle's operator
    res = f - oracle.apply_M(grid, x.cpu().numpy(), eta, mu)
    assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(f)
    s.close()


@pytest.mark.parametrize("smoother", ["jacobi", "hybrid"])
@pytest.mark.parametrize("dim,n,varmu", [(3, 16, False), (2, 32, True)])
def test_mg_gkb_matches_oracle(dim, n, varmu, smoother):
    """GKB with the MG-PCG inner solve against the oracle (Jacobi-PCG inner):
    both inner solves converged to 1e-13, so the GKB iterates agree."""
    _say("mg-gkb vs oracle", dim, n, varmu, smoother)
    gk = _gk()
    pr = P.stokes_problem(dim, n, seed=3, eta=1e2, lid=True, mu_seed=(7 if varmu else None))
    s = gk.Solver(pr.grid, pr.mu, pr.eta, inner="mg", inner_tol=1e-13, inner_maxit=50000,
                  smoother=smoother)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=1e-9, delay=5)
    ref = oracle.gkb_solve(pr.grid, pr.g, pr.r, pr.eta, mu=pr.mu, tol=1e-9, delay=5, maxit=300,
                           inner_tol=1e-13, inner_maxit=10 ** 6)
    assert info["iterations"] == ref["K"]
    assert _rel(w.cpu().numpy(), ref["w"]) <= 1e-8
    assert _rel(p.cpu().numpy(), ref["p"]) <= 1e-8
    s.close()


@pytest.mark.parametrize("dim,n,varmu,eta,smoother", [(3, 32, False, 1e3, "jacobi"),
                                                      (2, 64, True, 1e3, "jacobi"),
                                                      (3, 16, True, 1e2, "jacobi"),
                                                      (3, 32, False, 1e3, "hybrid"),
                                                      (2, 64, True, 1e3, "hybrid")])
def test_mixed_precision_residual(dim, n, varmu, eta, smoother):
    """FP32 inner MG-PCG inside FP64 GKB sweeps with FP64 defect correction:
    the FP64 saddle residual, recomputed by the oracle, is <= 1e-8; the
    difference to the oracle's FP64 solution is reported against it."""
    _say("mixed", dim, n, varmu, eta, smoother)
    gk = _gk()
    pr = P.stokes_problem(dim, n, seed=4, eta=eta, lid=(dim == 3), mu_seed=(8 if varmu else None))
    s = gk.Solver(pr.grid, pr.mu, pr.eta, precision="mixed", inner="mg", inner_tol=1e-5,
                  refine_tol=1e-8, max_sweeps=12, maxit=200, smoother=smoother)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=1e-4, delay=5)
    wn, pn = w.cpu().numpy(), p.cpu().numpy()
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, wn, pn, mu=pr.mu)
    assert nr[0] <= 1e-8 * nr[3], nr[0] / nr[3]
    assert info["residual"] <= 1e-8 and info["sweeps"] >= 2
    # library residual agrees with the oracle's
    assert abs(info["residual"] - nr[0] / nr[3]) <= 1e-6 * nr[0] / nr[3] + 1e-15
    s.close()


def test_fp64_mg_refinement_residual():
    _say("fp64 refine")
    gk = _gk()
    pr = P.stokes_problem(3, 32, seed=0, eta=1e3, lid=True)
    s = gk.Solver(pr.grid, None, pr.eta, inner="mg", inner_tol=1e-10, refine_tol=1e-8)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=1e-9, delay=5)
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w.cpu().numpy(), p.cpu().numpy())
    assert nr[0] <= 1e-8 * nr[3]
    s.close()


@pytest.mark.parametrize("dim,n,varmu", [(3, 32, False), (2, 128, False), (3, 24, True)])
def test_hybrid_smoother_robust_in_eta(dim, n, varmu):
    """At eta = 1e3 point-Jacobi multigrid leaves the divergence-free error of
    every level unsmoothed; the edge sweeps of the hybrid smoother remove it:
    at most a third of the MG-PCG iterations, edge weights on every level but
    the dense coarsest one."""
    _say("hybrid robustness", dim, n, varmu)
    gk = _gk()
    g = P.Grid(dim, (n, n, n if dim == 3 else 1), 1 / n, (D,) * 6, 0)
    mu = _mu(g, varmu)
    f = _dev(P.random_vector(g, 8))
    its = {}
    for sm in ("jacobi", "hybrid"):
        s = gk.Solver(g, mu, 1e3, inner="mg", smoother=sm, inner_maxit=20000)
        x, its[sm] = s.inner_solve(f, 1e-6)
        res = f.cpu().numpy() - oracle.apply_M(g, x.cpu().numpy(), 1e3, mu)
        assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(f.cpu().numpy())
        om = s.stats()["omega_edge"]
        if sm == "hybrid":
            assert all(v > 0 for v in om[:-1]) and om[-1] == 0.0, om
        else:
            assert all(v == 0.0 for v in om)
        s.close()
    assert 3 * its["hybrid"] <= its["jacobi"], its


def test_refinement_stops_when_a_sweep_does_not_reduce_the_residual():
    """Defect correction with inner solves far too loose for the sweep to
    converge: the solve ends with GKB_MAXIT (or GKB_OK), never above the
    initial residual, and the reported residual is that of the returned
    iterate."""
    _say("refinement guard")
    gk = _gk()
    pr = P.stokes_problem(3, 32, seed=0, eta=1e3, lid=True)
    s = gk.Solver(pr.grid, None, pr.eta, precision="mixed", inner="mg", inner_tol=0.3,
                  refine_tol=1e-12, max_sweeps=30, maxit=50)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=0.3, delay=1)
    assert info["status"] in (0, 1)
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w.cpu().numpy(), p.cpu().numpy())
    assert nr[0] <= nr[3]
    assert abs(info["residual"] - nr[0] / nr[3]) <= 1e-6 * nr[0] / nr[3]
    s.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_time_kernel_replays_and_leaves_the_solver_usable(prec):
    """gkb_time_kernel (graph replay of the finest-grid sweep, apply,
    residual and the two fused V-cycle sweeps) returns a positive time per
    launch, can be called repeatedly, and the next solve gives bitwise the
    same result as before."""
    _say("time kernel", prec)
    torch = __import__("torch")
    gk = _gk()
    pr = P.stokes_problem(3, 32, seed=2, eta=1e2)
    s = gk.Solver(pr.grid, None, pr.eta, inner="mg", precision=prec, inner_tol=1e-6,
                  refine_tol=1e-8, max_sweeps=10)
    g, r = _dev(pr.g), _dev(pr.r)
    w0, p0, _ = s.solve(g, r, tol=1e-3, delay=2)
    w0, p0 = w0.clone(), p0.clone()
    for k in ("smooth", "apply", "resid", "smooth_prolong", "smooth_zero", "smooth"):
        ms = s.time_kernel(k, 10)
        assert 0.0 < ms < 50.0, (k, ms)
    w1, p1, _ = s.solve(g, r, tol=1e-3, delay=2)
    torch.cuda.synchronize()
    assert torch.equal(w0, w1) and torch.equal(p0, p1)
    s.close()


def test_fp32_direction_update_fused_and_separate_agree():
    """FP32 MG-PCG forms the direction update inside the product when a
    captured chunk has an even number of iterations and runs the separate
    update kernel otherwise (odd chunk, 5): the same arithmetic, so the same
    iteration count and solution; the true residual of an FP32 solve sits at
    the FP32 level of this grad-div-dominated operator (eta = 1e3), above
    the recursive residual that stops it."""
    _say("fp32 direction update")
    gk = _gk()
    pr = P.stokes_problem(3, 32, seed=6, eta=1e3)
    f = _dev(pr.g)
    out = []
    for chunk in (8, 5):
        s = gk.Solver(pr.grid, None, pr.eta, inner="mg", precision="mixed", check_every=chunk)
        x, it = s.inner_solve(f, 1e-5)
        r = s.apply("M", x) - f
        out.append((x.cpu().numpy(), it, float((r * r).sum().sqrt() / (f * f).sum().sqrt())))
        s.close()
    (xa, ia, ra), (xb, ib, rb) = out
    assert ra <= 1e-3 and rb <= 1e-3, (ra, rb)
    assert ia == ib, (ia, ib)
    assert _rel(xa, xb) <= 1e-6
