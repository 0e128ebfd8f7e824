"""The configured workloads at full size.  The oracle cannot run the full
GKB solves (hours of Jacobi-PCG), so the checks are ones it can do at any
size: the FP64 saddle residual of the GPU answer recomputed by the oracle's
operators, element-wise operator parity on random vectors, and V-cycle
symmetry.  The 3D 128^3 case uses exactly the solver settings bench.py
times."""
import numpy as np
import pytest

import oracle
import problems as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(x, dtype=None):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype or torch.float64, device="cuda")


def _gk():
    import paper_2001_10424_amd as gk
    return gk


def _bench_modes():
    """The timed MG modes with the settings bench.py times them with
    (precision, inner, per-sweep lower-bound tolerance, inner tolerance,
    delay, smoother, sweeps)."""
    import bench  # the repository root is on sys.path (tests/conftest.py)
    out = {}
    for mode in ("fp64_mg", "mixed_mg", "fp64_gkb1", "fp64_mg_hybrid", "mixed_mg_hybrid"):
        prec, inner, tol, itol, delay, smoother, nu = bench.MODES[mode]
        out[mode] = dict(precision=prec, inner=inner, inner_tol=itol, tol=tol, delay=delay,
                         smoother=smoother, nu_pre=nu, nu_post=nu)
    return out


BENCH_MODES = _bench_modes()


def _solve(pr, mode):
    gk = _gk()
    m = dict(BENCH_MODES[mode])
    tol, delay = m.pop("tol"), m.pop("delay")
    kw = dict(inner_maxit=5000, maxit=200, refine_tol=1e-8, max_sweeps=30, check_every=8)
    kw.update(m)
    s = gk.Solver(pr.grid, pr.mu, pr.eta, **kw)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=tol, delay=delay)
    out = w.cpu().numpy(), p.cpu().numpy(), info
    s.close()
    return out


@pytest.mark.parametrize("mode", list(BENCH_MODES))
def test_stokes3d_128_lid_bench_config(mode):
    """The benchmarked workload: FP64 residual <= 1e-8 by the oracle."""
    _say("stokes3d_128_lid", mode)
    pr = P.stokes_problem(3, 128, seed=0, eta=1e3, lid=True)
    w, p, info = _solve(pr, mode)
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w, p)
    assert nr[0] <= 1e-8 * nr[3], nr[0] / nr[3]
    assert abs(info["residual"] - nr[0] / nr[3]) <= 1e-6 * nr[0] / nr[3] + 1e-15
    assert info["mg_levels"] == 5
    # pinned cell and non-unknown faces are zero
    assert p[0] == 0.0 and np.all(w[pr.grid.face_mask() == 0] == 0.0)


def test_stokes3d_128_lid_bench_config_learned():
    """The benchmarked value mode (FP32 inner flexible CG with V-cycle + CNN
    correction, MG-PCG fallback), with the network trained by bench.py's own
    recipe (pairs from forcing seed 1000, 64^3 crops): FP64 residual <= 1e-8
    by the oracle, and the statistics say which preconditioner carried the
    inner solves."""
    _say("stokes3d_128_lid mixed_learned")
    import torch

    import bench  # the repository root is on sys.path (tests/conftest.py)
    gk = _gk()
    net, train_info = bench.train_cnn(gk, torch, P, 128)
    pr = P.stokes_problem(3, 128, seed=0, eta=1e3, lid=True)
    s = bench.make_solver(gk, pr, "mixed_learned", net)
    tol, delay = bench.MODES["mixed_learned"][2], bench.MODES["mixed_learned"][4]
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=tol, delay=delay)
    s.close()
    w, p = w.cpu().numpy(), p.cpu().numpy()
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w, p)
    print("[case] learned_solves", info["learned_solves"], "fallbacks", info["fallbacks"],
          "gain", info["learned_gain"], "reason", info["learned_fallback_reason"],
          "inner", info["inner_iterations"], "train", train_info, flush=True)
    assert nr[0] <= 1e-8 * nr[3], nr[0] / nr[3]
    assert abs(info["residual"] - nr[0] / nr[3]) <= 1e-6 * nr[0] / nr[3] + 1e-15
    assert info["learned_solves"] >= 1
    assert p[0] == 0.0 and np.all(w[pr.grid.face_mask() == 0] == 0.0)


def test_stokes3d_128_operators_full_size():
    _say("operators 128^3")
    import torch
    gk = _gk()
    g = P.Grid(3, (128, 128, 128), 1 / 128, (P.DIRICHLET,) * 6, 0)
    s = gk.Solver(g, None, 1e3, inner="mg", precision="mixed")
    x = P.random_vector(g, 3)
    ref = oracle.apply_M(g, x, 1e3)
    y64 = s.apply("M", _dev(x)).cpu().numpy()
    assert np.abs(y64 - ref).max() <= 1e-13 * np.abs(ref).max()
    y32 = s.apply("M", _dev(x, torch.float32), precision="mixed").cpu().numpy()
    assert np.abs(y32 - ref).max() <= 3e-6 * np.abs(ref).max()
    # the FP32 V-cycle of the benchmarked hierarchy is symmetric
    a = _dev(P.random_vector(g, 4), torch.float32)
    b = _dev(P.random_vector(g, 5), torch.float32)
    va, vb = s.precondition(a, "mixed"), s.precondition(b, "mixed")
    l, r = float((a.double() * vb.double()).sum()), float((b.double() * va.double()).sum())
    assert abs(l - r) <= 1e-5 * abs(l)
    s.close()


@pytest.mark.parametrize("eta", [1e1, 1e3])
def test_stokes2d_512(eta):
    _say("stokes2d_512", eta)
    pr = P.stokes_problem(2, 512, seed=1, eta=eta)
    w, p, info = _solve(pr, "mixed_mg")
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w, p)
    assert nr[0] <= 1e-8 * nr[3]
    if eta == 1e1:
        # FP64 row of the configuration: parity with the mixed solution at
        # the level the residual target allows
        w2, p2, _ = _solve(pr, "fp64_mg")
        _, _, nr2 = oracle.saddle_residual(pr.grid, pr.g, pr.r, w2, p2)
        assert nr2[0] <= 1e-8 * nr2[3]
        assert np.linalg.norm(w - w2) <= 1e-6 * np.linalg.norm(w2)


@pytest.mark.parametrize("dim,n,mu_seed", [(2, 256, 7), (3, 192, 8)])
def test_varvisc_full_size_operators(dim, n, mu_seed):
    """Variable-viscosity workloads (contrast 1e3) at full size: the FP64 and
    FP32 operators against the oracle element-wise, and the symmetry of the
    V-cycle of the full hierarchy."""
    _say("varvisc operators", dim, n)
    import torch
    gk = _gk()
    pr = P.stokes_problem(dim, n, seed=10000, eta=1e3, mu_seed=mu_seed)
    assert abs(pr.mu.max() / pr.mu.min() - 1e3) <= 1e-6 * 1e3
    s = gk.Solver(pr.grid, pr.mu, pr.eta, inner="mg", precision="mixed")
    assert s.stats()["mg_levels"] == (6 if dim == 3 else 5)
    x = P.random_vector(pr.grid, 3)
    ref = oracle.apply_M(pr.grid, x, pr.eta, pr.mu)
    y = s.apply("M", _dev(x)).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    y32 = s.apply("M", _dev(x, torch.float32), precision="mixed").cpu().numpy()
    assert np.abs(y32 - ref).max() <= 3e-6 * np.abs(ref).max()
    a = _dev(P.random_vector(pr.grid, 4), torch.float32)
    b = _dev(P.random_vector(pr.grid, 5), torch.float32)
    va, vb = s.precondition(a, "mixed"), s.precondition(b, "mixed")
    l, r = float((a.double() * vb.double()).sum()), float((b.double() * va.double()).sum())
    assert abs(l - r) <= 1e-5 * abs(l)
    s.close()


@pytest.mark.parametrize("dim,n,mu_seed", [(2, 128, 7), (3, 48, 8)])
def test_varvisc_reduced_solve(dim, n, mu_seed):
    """Full mixed-precision solves of the variable-viscosity problems at
    reduced size (point-Jacobi multigrid needs many iterations at contrast
    1e3 with eta = 1e3): FP64 residual <= 1e-8 by the oracle."""
    _say("varvisc reduced solve", dim, n)
    gk = _gk()
    pr = P.stokes_problem(dim, n, seed=10000, eta=1e3, mu_seed=mu_seed)
    s = gk.Solver(pr.grid, pr.mu, pr.eta, precision="mixed", inner="mg", inner_tol=1e-3,
                  inner_maxit=100000, maxit=200, refine_tol=1e-8, max_sweeps=30)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=1e-2, delay=2)
    print("[case] sweeps", info["sweeps"], "inner", info["inner_iterations"], flush=True)
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w.cpu().numpy(), p.cpu().numpy(),
                                      mu=pr.mu)
    assert nr[0] <= 1e-8 * nr[3]
    s.close()


@pytest.mark.parametrize("dim,n,mu_seed", [(2, 256, 7), (3, 192, 8)])
def test_varvisc_full_size_solve_hybrid(dim, n, mu_seed):
    """The variable-viscosity workloads (log-normal mu, contrast 1e3, eta =
    1e3) at full size with FP32 inner MG-PCG on the hybrid face + edge
    smoother (point-Jacobi multigrid needs thousands of iterations per inner
    solve here), with the per-sweep setting of the timed hybrid mode: FP64
    residual <= 1e-8 by the oracle."""
    _say("varvisc full solve hybrid", dim, n)
    gk = _gk()
    m = BENCH_MODES["mixed_mg_hybrid"]
    pr = P.stokes_problem(dim, n, seed=10000, eta=1e3, mu_seed=mu_seed)
    s = gk.Solver(pr.grid, pr.mu, pr.eta, precision="mixed", inner="mg", smoother="hybrid",
                  nu_pre=1, nu_post=1, inner_tol=m["inner_tol"], inner_maxit=20000, maxit=200,
                  refine_tol=1e-8, max_sweeps=30)
    w, p, info = s.solve(_dev(pr.g), _dev(pr.r), tol=m["tol"], delay=m["delay"])
    print("[case] sweeps", info["sweeps"], "K", info["outer_iterations"], "inner",
          info["inner_iterations"], flush=True)
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, w.cpu().numpy(), p.cpu().numpy(),
                                      mu=pr.mu)
    assert nr[0] <= 1e-8 * nr[3]
    assert info["mg_levels"] == (6 if dim == 3 else 5)
    s.close()
