"""Writes the golden fixtures of this folder from closed forms the paper
prints (no solver is run):

poiseuille_s41_<nx>x<ny>.txt -- the exact Poiseuille flow of Section 4.1
(Poiseuille Flow) of arXiv 2001.10424: channel [0, 2] x [0, 1], velocity
(4y(1-y), 0) and pressure 8(2-x), sampled at the MAC locations of an
nx x ny grid (u at the x-faces (i h, (j + 1/2) h), p at the cell centres).

    python tests/golden/make_fixtures.py
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def poiseuille(nx, ny, length=2.0):
    h = 1.0 / ny
    lines = [
        "# arXiv 2001.10424, Section 4.1 (Poiseuille Flow): exact solution of the 2D Stokes",
        "# problem -Laplace(u) + grad(p) = 0, div(u) = 0 on the channel [0, 2] x [0, 1]:",
        "# u(x, y) = (4 y (1 - y), 0), p(x, y) = 8 (2 - x).",
        f"# sampled on the MAC grid nx = {nx}, ny = {ny}, h = 1/{ny}: rows 'u i j value' at the",
        "# x-faces (i h, (j + 1/2) h), i = 0..nx; rows 'p i j value' at the cell centres.",
        f"grid {nx} {ny} {length}",
    ]
    for j in range(ny):
        y = (j + 0.5) * h
        for i in range(nx + 1):
            lines.append(f"u {i} {j} {4.0 * y * (1.0 - y):.17g}")
    for j in range(ny):
        for i in range(nx):
            x = (i + 0.5) * h
            lines.append(f"p {i} {j} {8.0 * (length - x):.17g}")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    for nx, ny in ((16, 8), (32, 16)):
        with open(os.path.join(HERE, f"poiseuille_s41_{nx}x{ny}.txt"), "w") as f:
            f.write(poiseuille(nx, ny))
