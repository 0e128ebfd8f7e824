"""Pins of the oracle's MAC operators (W, A, A^T, M, diag M) against facts that
do not come from the oracle itself: symmetry, adjointness, definiteness, rank,
exactness on polynomials, flux balance for piecewise-constant viscosity and
O(h^2) convergence to the paper's Poiseuille solution (Section 4.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
import problems as P

D, N = P.DIRICHLET, P.NATURAL

GRIDS = [
    P.Grid(2, (6, 4, 1), 0.25, (D, N, D, D, D, D), -1),   # channel: outflow at +x
    P.Grid(2, (5, 5, 1), 0.2, (D,) * 6, 0),               # box, pinned cell
    P.Grid(3, (4, 3, 5), 0.2, (D,) * 6, 0),
    P.Grid(3, (3, 4, 3), 0.25, (D, N, D, D, N, D), -1),   # two natural sides
]


def _mu(g, seed=3):
    return np.exp(np.random.default_rng(seed).standard_normal(g.n_cells))


def _sub(g):
    return g.face_mask() > 0, g.cell_mask() > 0


def test_layout_sizes_match_generator():
    for g in GRIDS:
        m, n = oracle.sizes(g)
        assert m == g.m_full and n == g.n_cells


@pytest.mark.parametrize("gi", range(len(GRIDS)))
@pytest.mark.parametrize("varmu", [False, True])
def test_W_symmetric_positive_definite(gi, varmu):
    g = GRIDS[gi]
    mu = _mu(g) if varmu else None
    fm, _ = _sub(g)
    W = oracle.dense(g, "W", mu=mu)
    # rows and columns of non-unknown faces are zero
    assert np.all(W[~fm] == 0) and np.all(W[:, ~fm] == 0)
    Wu = W[np.ix_(fm, fm)]
    assert np.abs(Wu - Wu.T).max() <= 1e-13 * np.abs(Wu).max()
    assert np.linalg.eigvalsh(Wu).min() > 0


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_AT_is_adjoint_and_A_full_rank(gi):
    g = GRIDS[gi]
    fm, cm = _sub(g)
    A = oracle.dense(g, "A")
    AT = oracle.dense(g, "AT")
    assert np.array_equal(A, AT.T)
    Au = A[np.ix_(fm, cm)]
    sv = np.linalg.svd(Au, compute_uv=False)
    assert sv.min() > 1e-8 * sv.max()
    # random-vector adjointness y.(A p) = (A^T y).p
    y = P.random_vector(g, 1)
    p = P.random_vector(g, 2, "cells")
    lhs = y @ oracle.apply_A(g, p)
    rhs = oracle.apply_AT(g, y) @ p
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_M_is_W_plus_eta_AAT_and_diag(gi):
    g = GRIDS[gi]
    mu = _mu(g)
    for eta in (0.0, 10.0, 1e3):
        W = oracle.dense(g, "W", mu=mu)
        A = oracle.dense(g, "A")
        M = oracle.dense(g, "M", eta=eta, mu=mu)
        ref = W + eta * A @ A.T
        assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()
        d = oracle.diag_M(g, eta, mu)
        assert np.abs(d - np.diag(ref)).max() <= 1e-12 * np.abs(ref).max()


def test_random_vector_symmetry_3d_varmu():
    g = P.Grid(3, (8, 6, 7), 1 / 8, (D,) * 6, 0)
    mu = _mu(g)
    x = P.random_vector(g, 5)
    y = P.random_vector(g, 6)
    a = x @ oracle.apply_M(g, y, 100.0, mu)
    b = y @ oracle.apply_M(g, x, 100.0, mu)
    assert abs(a - b) <= 1e-13 * abs(a)


def _interior_faces(g, depth=1):
    """Faces whose whole 7-point neighbourhood stays away from every wall."""
    keep = np.zeros(g.m_full, dtype=bool)
    for c, comp in enumerate(g.split(keep)):
        idx = np.indices(comp.shape)  # (z, y, x)
        ok = np.ones(comp.shape, dtype=bool)
        for a in range(g.dim):
            ax = 2 - a
            lim = comp.shape[ax]
            ok &= (idx[ax] >= depth + 1) & (idx[ax] <= lim - depth - 2)
        comp[...] = ok
    return keep


def test_polynomial_exactness_2d():
    """Second differences are exact on cubics, and the MAC gradient is exact on
    quadratics: at faces away from walls W u + A p equals the continuous
    -Lap u + grad p for the paper's 2D solution (Section 4.2)."""
    n = 16
    g = P.Grid(2, (n, n, 1), 1.0 / n, (D,) * 6, -1)
    w, p = P.polynomial_2d_fields(g)
    lhs = oracle.apply_W_ext(g, w) + oracle.apply_A(g, p)
    f = np.zeros(g.m_full)
    X, Y = g.face_centres(0)
    g.split(f)[0][:] = -3 * X - 6 * Y
    X, Y = g.face_centres(1)
    g.split(f)[1][:] = -12 * X + 9 * Y
    keep = _interior_faces(g)
    assert keep.sum() > 100
    assert np.abs(lhs - f)[keep].max() <= 1e-9
    # A^T = -div: the central difference of the cubic u in x is 3x^2 + h^2/4,
    # that of v in y is -3x^2, so A^T w = -h^2/4 in every cell not touching a
    # wall (A^T ignores the prescribed wall-normal faces)
    t = oracle.apply_AT(g, w).reshape(n, n)
    assert np.abs(t[1:-1, 1:-1] + g.h ** 2 / 4).max() <= 1e-12


def test_polynomial_exactness_3d():
    """3D cubic field of the paper (Section 4.4), exact interior stencil."""
    n = 12
    g = P.Grid(3, (n, n, n), 1.0 / n, (D,) * 6, -1)
    w = np.zeros(g.m_full)
    comps = g.split(w)
    X, Y, Z = g.face_centres(0)
    comps[0][:] = X ** 3 + Y ** 3 + 3 * Z ** 2 * X
    X, Y, Z = g.face_centres(1)
    comps[1][:] = 2 * X ** 3 - 3 * X ** 2 * Y
    X, Y, Z = g.face_centres(2)
    comps[2][:] = -Z ** 3 * X + Y ** 2
    Xc, Yc, Zc = g.cell_centres()
    p = (1.5 * (Xc ** 2 + Yc ** 2 + Zc ** 2) - 1.5).reshape(-1)
    lhs = oracle.apply_W_ext(g, w) + oracle.apply_A(g, p)
    f = np.zeros(g.m_full)
    fc = g.split(f)
    X, Y, Z = g.face_centres(0)   # -Lap u + p_x
    fc[0][:] = -(6 * X + 6 * Y + 6 * X) + 3 * X
    X, Y, Z = g.face_centres(1)
    fc[1][:] = -(12 * X - 6 * Y) + 3 * Y
    X, Y, Z = g.face_centres(2)
    fc[2][:] = -(-6 * Z * X + 2) + 3 * Z
    keep = _interior_faces(g)
    assert np.abs(lhs - f)[keep].max() <= 1e-8


def test_variable_viscosity_flux_balance():
    """Piecewise-constant viscosity varying along one axis: a field whose
    discrete flux mu * du/dn is constant has zero W-image at interior faces.
    This fixes where cell and edge viscosities enter: normal couplings use the
    cell between the faces, tangential couplings the mean over the cells that
    touch the edge (for mu(y) the two cells below/above the edge)."""
    nx, ny = 6, 9
    g = P.Grid(2, (nx, ny, 1), 1.0 / ny, (D,) * 6, -1)
    rng = np.random.default_rng(4)
    # (1) normal direction: mu = mu(x), u(x) with mu_i (u_{i+1} - u_i) = const
    mux = np.exp(rng.standard_normal(nx))
    mu = np.tile(mux, (ny, 1)).reshape(-1)
    u_line = np.concatenate([[0.0], np.cumsum(1.0 / mux)])
    w = np.zeros(g.m_full)
    g.split(w)[0][0][:] = u_line[None, :]
    y = oracle.apply_W_ext(g, w, mu=mu)
    uy = g.split(y)[0][0]
    assert np.abs(uy[1:-1, 1:-1]).max() <= 1e-10
    # (2) tangential direction: mu = mu(y); the edge between rows j and j+1
    # has mu_e = (mu_j + mu_{j+1}) / 2 at interior vertices
    muy = np.exp(rng.standard_normal(ny))
    mu = np.repeat(muy, nx).reshape(-1)
    mue = 0.5 * (muy[:-1] + muy[1:])
    col = np.concatenate([[0.0], np.cumsum(1.0 / mue)])
    w = np.zeros(g.m_full)
    g.split(w)[0][0][:] = col[:, None]
    y = oracle.apply_W_ext(g, w, mu=mu)
    uy = g.split(y)[0][0]
    assert np.abs(uy[1:-1, 2:-2]).max() <= 1e-9


def test_mu_one_equals_isoviscous_and_scales():
    g = GRIDS[2]
    x = P.random_vector(g, 9)
    a = oracle.apply_W(g, x)
    b = oracle.apply_W(g, x, mu=np.ones(g.n_cells))
    c = oracle.apply_W(g, x, mu=3.0 * np.ones(g.n_cells))
    assert np.array_equal(a, b)
    assert np.allclose(c, 3.0 * a, rtol=1e-14, atol=0)


def test_lid_rhs_matches_moving_wall():
    """The closed-form lid term of the input generator equals the change of W
    applied to a field at rest when the top wall moves with u = 1."""
    for g in (P.Grid(2, (8, 8, 1), 1 / 8, (D,) * 6, 0), P.Grid(3, (6, 6, 6), 1 / 6, (D,) * 6, 0)):
        top = 3 if g.dim == 2 else 5
        wall = np.zeros((6, 3))
        wall[top, 0] = 1.0
        zero = np.zeros(g.m_full)
        y = oracle.apply_W_ext(g, zero, wall_tan=wall)
        assert np.abs(-y * g.face_mask() - P.lid_rhs(g, 1.0)).max() <= 1e-9


def test_poiseuille_rhs_is_lifted_boundary_data():
    """g of the Poiseuille fixture is -W_ext applied to the lifted inflow."""
    pr = P.poiseuille_problem(64, 16, 4.0, 1e2)
    g = pr.grid
    y = oracle.apply_W_ext(g, pr.extra["w_lift"])
    assert np.abs(-y * g.face_mask() - pr.g).max() <= 1e-10


def _direct(pr):
    g = pr.grid
    fm, cm = _sub(g)
    W = sp.csr_matrix(oracle.dense(g, "W", mu=pr.mu)[np.ix_(fm, fm)])
    A = sp.csr_matrix(oracle.dense(g, "A")[np.ix_(fm, cm)])
    K = sp.bmat([[W, A], [A.T, None]]).tocsc()
    sol = spl.spsolve(K, np.concatenate([pr.g[fm], pr.r[cm]]))
    w = np.zeros(g.m_full)
    p = np.zeros(g.n_cells)
    w[fm] = sol[:fm.sum()]
    p[cm] = sol[fm.sum():]
    return w, p


def test_poiseuille_second_order_convergence():
    """Discrete Poiseuille solutions converge to u = 4y(1-y), p = 8(L-x) at
    O(h^2) in the RMS norm (paper Section 4.1, channel lengthened to L = 4)."""
    errs = []
    for ny in (8, 16, 32):
        pr = P.poiseuille_problem(4 * ny, ny, 4.0, 1e2)
        w, p = _direct(pr)
        g = pr.grid
        eu = (pr.extra["w_lift"] + w - pr.extra["u_exact"]) * g.face_mask()
        ep = p - pr.extra["p_exact"]
        errs.append((np.sqrt(np.mean(eu ** 2)), np.sqrt(np.mean(ep ** 2))))
    for (u0, p0), (u1, p1) in zip(errs[:-1], errs[1:]):
        assert u0 / u1 >= 3.5 and p0 / p1 >= 3.5, errs
    # the interior rows of the coarsest channel solve the momentum balance of
    # the exact linear pressure exactly: outflow pressure p_{N-1} = 4 h
    assert errs[-1][0] < 1e-3 and errs[-1][1] < 0.05


def test_layout_and_masks():
    g = P.Grid(2, (64, 16, 1), 1 / 16, (D, N, D, D, D, D), -1)
    assert g.m == 64 * 16 + 64 * 15 and g.n_p == 1024
    g = P.Grid(3, (128, 128, 128), 1 / 128, (D,) * 6, 0)
    assert g.m == 6242304 and g.n_p == 2097151
