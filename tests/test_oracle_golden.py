"""The oracle against the paper's printed exact solution (golden fixtures in
tests/golden/, written by make_fixtures.py from Section 4.1): the discrete
Poiseuille flow on the paper's channel [0, 2] x [0, 1], solved by the
oracle's GKB with Jacobi-PCG, lies within O(h^2) of the fixture values (in
the mean) and the error falls by about 4 when h halves."""
import os

import numpy as np
import pytest

import oracle
import problems as P

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    u, p, grid = {}, {}, None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "grid":
                grid = (int(parts[1]), int(parts[2]), float(parts[3]))
            elif parts[0] == "u":
                u[(int(parts[1]), int(parts[2]))] = float(parts[3])
            else:
                p[(int(parts[1]), int(parts[2]))] = float(parts[3])
    return grid, u, p


def _errors(name):
    (nx, ny, length), u_ex, p_ex = _load(name)
    pr = P.poiseuille_problem(nx, ny, length, 1e2)
    res = oracle.gkb_solve(pr.grid, pr.g, pr.r, pr.eta, tol=1e-12, delay=5, maxit=500,
                           inner_tol=1e-13, inner_maxit=10 ** 6)
    assert res["status"] == 0
    g = pr.grid
    u = g.split(pr.extra["w_lift"] + res["w"])[0][0]      # (ny, nx + 1) incl. inflow
    p = res["p"].reshape(ny, nx)
    du = np.array([u[j, i] - v for (i, j), v in u_ex.items()])
    dp = np.array([p[j, i] - v for (i, j), v in p_ex.items()])
    assert len(du) == ny * (nx + 1) and len(dp) == nx * ny
    rms = lambda d: float(np.sqrt(np.mean(d * d)))
    return float(np.abs(du).max()), rms(du), rms(dp), 1.0 / ny


def test_poiseuille_matches_the_papers_exact_solution():
    m1u, e1u, e1p, h1 = _errors("poiseuille_s41_16x8.txt")
    m2u, e2u, e2p, h2 = _errors("poiseuille_s41_32x16.txt")
    # second order in the mean (the mirrored ghost at the no-slip walls is the
    # O(h^2) term); the pressure's largest error sits at the inflow corners
    # and converges more slowly, so it is bounded in the mean only
    assert m1u <= 1.2 * h1 ** 2 and m2u <= 1.2 * h2 ** 2, (m1u, m2u)
    assert e1u <= 0.6 * h1 ** 2 and e2u <= 0.6 * h2 ** 2, (e1u, e2u)
    assert e1p <= 20.0 * h1 ** 2 and e2p <= 20.0 * h2 ** 2, (e1p, e2p)
    assert e1u / e2u >= 3.5 and e1p / e2p >= 3.5, (e1u / e2u, e1p / e2p)
