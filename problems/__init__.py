"""Seeded synthetic inputs for the MAC-grid Stokes saddle-point problems.

This module holds only input generation: grid descriptions, body forces,
boundary data folded into the right-hand side in closed form, viscosity
fields and random manufactured solutions.  It contains none of the solver's
arithmetic (no operator application, no Krylov or GKB step) and it is the only
code shared by the CPU oracle (``oracle/``) and the GPU library
(``paper_2001_10424_amd``).

Problem being solved (paper, Section 1, saddle-point system):

    [[W, A], [A^T, 0]] [w; p] = [g; r]

with W the (variable-viscosity) vector Laplacian and A the discrete gradient on
a staggered (MAC) grid.

Array layout (shared with the C-ABI, see ``include/gkb.h``):
  * velocity is stored full-face, component-major (structure of arrays):
    u[nz][ny][nx+1], then v[nz][ny+1][nx], then (3D) w[nz+1][ny][nx];
    x is the fastest index.  2D grids use nz = 1 and have no w block.
  * pressure and the second right-hand side r live on cells [nz][ny][nx].
  * faces normal to a DIRICHLET boundary are not unknowns; their entries are 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

DIRICHLET = 0
NATURAL = 1


@dataclass(frozen=True)
class Grid:
    """Uniform MAC grid.  ``bc`` lists the boundary type of the sides
    -x, +x, -y, +y, -z, +z.  ``pin`` is the flat index of a cell whose
    pressure is fixed to 0 (removed from the unknowns), or -1."""

    dim: int
    n: tuple
    h: float
    bc: tuple = (DIRICHLET,) * 6
    pin: int = -1

    @property
    def nx(self):
        return self.n[0]

    @property
    def ny(self):
        return self.n[1]

    @property
    def nz(self):
        return self.n[2] if self.dim == 3 else 1

    def comp_shape(self, c):
        """(nz, ny, nx)-ordered shape of the face array of component c."""
        s = [self.nz, self.ny, self.nx]
        s[2 - c] += 1
        return tuple(s)

    @property
    def cell_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_cells(self):
        return self.nx * self.ny * self.nz

    def comp_size(self, c):
        return int(np.prod(self.comp_shape(c)))

    @property
    def m_full(self):
        return sum(self.comp_size(c) for c in range(self.dim))

    def offsets(self):
        off, o = [], 0
        for c in range(self.dim):
            off.append(o)
            o += self.comp_size(c)
        return off

    def split(self, x):
        """Views of a full-face vector as per-component (nz, ny, nx') arrays."""
        out = []
        for c, o in enumerate(self.offsets()):
            out.append(x[o:o + self.comp_size(c)].reshape(self.comp_shape(c)))
        return out

    def face_mask(self):
        """1.0 at unknown faces, 0.0 at faces normal to a DIRICHLET side."""
        mask = np.ones(self.m_full)
        for c, comp in enumerate(self.split(mask)):
            ax = 2 - c  # numpy axis of the normal index
            nn = comp.shape[ax]
            if self.bc[2 * c] == DIRICHLET:
                np.moveaxis(comp, ax, 0)[0] = 0.0
            if self.bc[2 * c + 1] == DIRICHLET:
                np.moveaxis(comp, ax, 0)[nn - 1] = 0.0
        return mask

    def cell_mask(self):
        mask = np.ones(self.n_cells)
        if self.pin >= 0:
            mask[self.pin] = 0.0
        return mask

    @property
    def m(self):
        return int(self.face_mask().sum())

    @property
    def n_p(self):
        return int(self.cell_mask().sum())

    def face_centres(self, c):
        """Coordinates (X, Y[, Z]) of the face centres of component c, each an
        array of the component's shape."""
        axes = []
        for a in range(self.dim):
            na = self.n[a]
            if a == c:
                axes.append(np.arange(na + 1) * self.h)
            else:
                axes.append((np.arange(na) + 0.5) * self.h)
        if self.dim == 2:
            Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
            return X[None], Y[None]
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        return X, Y, Z

    def cell_centres(self):
        axes = [(np.arange(self.n[a]) + 0.5) * self.h for a in range(self.dim)]
        if self.dim == 2:
            Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
            return X[None], Y[None]
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        return X, Y, Z


@dataclass
class Problem:
    """One saddle-point instance: right-hand sides, viscosity and the augmented
    Lagrangian parameter eta (the paper's nu; eta = 0 switches it off)."""

    name: str
    grid: Grid
    g: np.ndarray
    r: np.ndarray
    mu: np.ndarray | None
    eta: float
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# Body forces and viscosity fields
# ----------------------------------------------------------------------------

def fourier_forcing(grid: Grid, seed: int, modes: int = 8, kmax: int = 8):
    """Sum of ``modes`` random Fourier modes sampled at face centres:
    f_c(x) = sum_m a_{c,m} cos(2 pi k_m . x + phi_m), k_m integer in
    [1, kmax]^dim, phi_m ~ U[0, 2 pi), a ~ N(0, 1).  Draw order per mode:
    k_m, then phi_m, then the dim amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, phis, amps = [], [], []
    for _ in range(modes):
        ks.append(rng.integers(1, kmax + 1, size=grid.dim))
        phis.append(rng.uniform(0.0, 2.0 * math.pi))
        amps.append(rng.standard_normal(grid.dim))
    f = np.zeros(grid.m_full)
    for c, comp in enumerate(grid.split(f)):
        X = grid.face_centres(c)
        for k, phi, a in zip(ks, phis, amps):
            arg = sum(2.0 * math.pi * k[d] * X[d] for d in range(grid.dim)) + phi
            comp += a[c] * np.cos(arg)
    return f * grid.face_mask()


def lognormal_viscosity(grid: Grid, seed: int, corr_len: float = 0.1,
                        contrast: float = 1e3):
    """Log-normal viscosity on cells: white noise N(0,1) (PCG64(seed)),
    filtered periodically in Fourier space by exp(-corr_len^2 |k|^2 / 4) with
    angular wavenumbers k, standardised to G, then mu = exp(s G) with
    s = ln(contrast) / (max G - min G): max(mu)/min(mu) = contrast exactly and
    the geometric mean of mu is 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal(grid.cell_shape)
    F = np.fft.fftn(white)
    ks = [2.0 * math.pi * np.fft.fftfreq(s, d=grid.h) for s in grid.cell_shape]
    K = np.meshgrid(*ks, indexing="ij")
    k2 = sum(k * k for k in K)
    G = np.real(np.fft.ifftn(F * np.exp(-corr_len ** 2 * k2 / 4.0)))
    G = (G - G.mean()) / G.std()
    s = math.log(contrast) / (G.max() - G.min())
    return np.exp(s * G).reshape(-1)


# ----------------------------------------------------------------------------
# Boundary data folded into the right-hand side (closed forms)
# ----------------------------------------------------------------------------

def lid_rhs(grid: Grid, U: float = 1.0, mu: float = 1.0):
    """Moving lid: u = U on the top wall (+y in 2D, +z in 3D).  With the wall
    ghost value 2U - u_f of the viscous stencil, the wall term of the u-faces
    next to the lid contributes 2 mu_e U / h^2 to g.  Only u-faces that are
    unknowns get it; mu_e is the constant viscosity ``mu``."""
    g = np.zeros(grid.m_full)
    u = grid.split(g)[0]
    val = 2.0 * mu * U / grid.h ** 2
    if grid.dim == 3:
        u[grid.nz - 1, :, :] = val
    else:
        u[0, grid.ny - 1, :] = val
    return g * grid.face_mask()


def poiseuille_problem(nx=64, ny=16, length=4.0, eta=1e2):
    """Channel [0, length] x [0, 1], parabolic inflow u = 4y(1-y) at x = 0,
    no-slip at y = 0, 1, do-nothing outflow at x = length (paper, Section 4.1,
    with the channel lengthened).  h = 1/ny and nx = length * ny.

    The solve is for the correction w~ = w - w_b of the lifted field
    w_b = (4y(1-y), 0) sampled on all u-faces; w_b is discretely divergence
    free, so r = 0, and g = -W_ext w_b.  For the sampled parabola the
    y-second difference is exact in interior rows (-(u_{j+1}-2u_j+u_{j-1})/h^2
    = 8), while in the two wall rows the mirrored ghost -u_j gives
    (3 u_0 - u_1)/h^2 = 6 for every h.  Faces on the outflow boundary own half
    a control volume, which halves their tangential (y) terms; the x-terms of
    w_b vanish because it does not vary in x.  Hence g_u = -8, -6 (wall rows),
    halved on the outflow faces, and g_v = 0.

    Exact solution of the continuous problem: u = 4y(1-y), v = 0,
    p = 8(length - x)."""
    assert abs(nx - length * ny) < 1e-9
    grid = Grid(dim=2, n=(nx, ny, 1), h=1.0 / ny,
                bc=(DIRICHLET, NATURAL, DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET),
                pin=-1)
    g = np.zeros(grid.m_full)
    u = grid.split(g)[0][0]          # (ny, nx+1)
    u[:, :] = -8.0
    u[0, :] = -6.0
    u[ny - 1, :] = -6.0
    u[:, nx] *= 0.5
    g *= grid.face_mask()
    r = np.zeros(grid.n_cells)
    wb = np.zeros(grid.m_full)
    X, Y = grid.face_centres(0)
    grid.split(wb)[0][:] = 4.0 * Y * (1.0 - Y)
    Xc, _ = grid.cell_centres()
    u_exact = wb.copy()
    p_exact = (8.0 * (length - Xc)).reshape(-1)
    return Problem("poiseuille", grid, g, r, None, eta,
                   extra=dict(w_lift=wb, u_exact=u_exact, p_exact=p_exact))


# ----------------------------------------------------------------------------
# Manufactured solutions
# ----------------------------------------------------------------------------

def random_solution(grid: Grid, seed: int):
    """Random (w*, p*) with N(0,1) entries on the unknowns (PCG64(seed)):
    first all face entries, then all cell entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(grid.m_full) * grid.face_mask()
    p = rng.standard_normal(grid.n_cells) * grid.cell_mask()
    return w, p


def random_vector(grid: Grid, seed: int, where="faces"):
    rng = np.random.Generator(np.random.PCG64(seed))
    if where == "faces":
        return rng.standard_normal(grid.m_full) * grid.face_mask()
    return rng.standard_normal(grid.n_cells) * grid.cell_mask()


def polynomial_2d_fields(grid: Grid):
    """Exact 2D Stokes solution of the paper's Section 4.2:
    u = (x^3 + y^3, 2x^3 - 3x^2 y), p = 1.5x^2 + 1.5y^2 - 1, sampled at face /
    cell centres (including boundary faces)."""
    w = np.zeros(grid.m_full)
    X, Y = grid.face_centres(0)
    grid.split(w)[0][:] = X ** 3 + Y ** 3
    X, Y = grid.face_centres(1)
    grid.split(w)[1][:] = 2 * X ** 3 - 3 * X ** 2 * Y
    Xc, Yc = grid.cell_centres()
    p = (1.5 * Xc ** 2 + 1.5 * Yc ** 2 - 1.0).reshape(-1)
    return w, p


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def stokes_problem(dim, n, seed=0, eta=1e3, lid=False, mu_seed=None,
                   contrast=1e3, corr_len=0.1):
    """Unit square / cube, no-slip walls on all sides, pressure pinned at
    cell 0, 8-mode Fourier body force (seed), optional lid u = 1 on the top
    wall, optional log-normal viscosity (mu_seed)."""
    nn = (n, n, n if dim == 3 else 1)
    grid = Grid(dim=dim, n=nn, h=1.0 / n, bc=(DIRICHLET,) * 6, pin=0)
    g = fourier_forcing(grid, seed)
    if lid:
        g = g + lid_rhs(grid, 1.0, 1.0)
    mu = None
    if mu_seed is not None:
        mu = lognormal_viscosity(grid, mu_seed, corr_len, contrast)
    r = np.zeros(grid.n_cells)
    name = f"stokes{dim}d_{n}" + ("_lid" if lid else "") + ("_varmu" if mu is not None else "")
    return Problem(name, grid, g, r, mu, eta, extra=dict(seed=seed))


WORKLOADS = {
    # 2D Poiseuille channel, 64 x 16 cells on [0,4] x [0,1], eta = 1e2
    "poiseuille_64x16": lambda seed=0: poiseuille_problem(64, 16, 4.0, 1e2),
    # 2D isoviscous Stokes 512^2, 8-mode forcing, eta in {1e1, 1e3}
    "stokes2d_512": lambda seed=0, eta=1e3: stokes_problem(2, 512, seed, eta),
    # 3D isoviscous lid-driven Stokes 128^3 + 8-mode forcing, eta = 1e3
    "stokes3d_128_lid": lambda seed=0: stokes_problem(3, 128, seed, 1e3, lid=True),
    # 2D variable viscosity 256^2, log-normal mu (seed 7), eta = 1e3
    "varvisc2d_256": lambda seed=0: stokes_problem(2, 256, seed, 1e3, mu_seed=7),
    # 3D variable viscosity 192^3, log-normal mu (seed 8), eta = 1e3
    "varvisc3d_192": lambda seed=0: stokes_problem(3, 192, seed, 1e3, mu_seed=8),
}
