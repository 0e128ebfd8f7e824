"""CPU FP64 oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C, FP64,
OpenMP) through ctypes and ``cnn_ref.py`` (NumPy CNN reference).  It shares
no code with the GPU library ``paper_2001_10424_amd``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, MAXIT, EINVAL, ENOMEM, ENAN, EINNER = 0, 1, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double),
                ("bc", C.c_int * 6), ("pin", C.c_int)]


class _GkbOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("delay", C.c_int), ("maxit", C.c_int),
                ("inner_tol", C.c_double), ("inner_maxit", C.c_int),
                ("squared_rule", C.c_int),
                ("zeta", C.c_void_p), ("alpha", C.c_void_p), ("beta", C.c_void_p),
                ("est_hist", C.c_void_p), ("inner_iters", C.c_void_p),
                ("store_k", C.c_int), ("V", C.c_void_p), ("Q", C.c_void_p),
                ("inner_krylov", C.c_int), ("restart", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        G = C.POINTER(_Grid)
        L.og_m_full.argtypes = [G]
        L.og_m_full.restype = C.c_long
        L.og_n_cells.argtypes = [G]
        L.og_n_cells.restype = C.c_long
        L.og_apply_W.argtypes = [G, P, P, P]
        L.og_apply_W_ext.argtypes = [G, P, P, P, P]
        L.og_apply_A.argtypes = [G, P, P]
        L.og_apply_AT.argtypes = [G, P, P]
        L.og_apply_M.argtypes = [G, P, C.c_double, P, P]
        L.og_diag_M.argtypes = [G, P, C.c_double, P]
        L.og_pcg.argtypes = [G, P, C.c_double, P, P, C.c_double, C.c_int,
                             C.POINTER(C.c_int)]
        L.og_pcg.restype = C.c_int
        L.og_gkb_solve.argtypes = [G, P, C.c_double, P, P, C.POINTER(_GkbOpts), P, P,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double),
                                   C.POINTER(C.c_int)]
        L.og_gkb_solve.restype = C.c_int
        L.og_saddle_residual.argtypes = [G, P, P, P, P, P, P, P, P]
        L.og_gkb_fgmres.argtypes = [G, P, C.c_double, P, P, C.POINTER(_GkbOpts), C.c_double,
                                    C.c_int, C.c_int, P, P, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
        L.og_gkb_fgmres.restype = C.c_int
        L.og_csr_central_scaling.argtypes = [C.c_int, C.c_int] + [P] * 8
        L.og_csr_central_scaling.restype = C.c_int
        L.og_gkb_solve_csr.argtypes = [C.c_int, C.c_int] + [P] * 6 + [C.c_double, C.c_int, P, P,
                                       C.POINTER(_GkbOpts), P, P, C.POINTER(C.c_int),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.og_gkb_solve_csr.restype = C.c_int
        _lib = L
    return _lib


def _grid(grid) -> _Grid:
    gs = _Grid()
    gs.dim = grid.dim
    for a in range(3):
        gs.n[a] = int(grid.n[a]) if a < grid.dim else 1
    gs.h = float(grid.h)
    for s in range(6):
        gs.bc[s] = int(grid.bc[s])
    gs.pin = int(grid.pin)
    return gs


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def sizes(grid):
    gs = _grid(grid)
    return lib().og_m_full(C.byref(gs)), lib().og_n_cells(C.byref(gs))


def apply_W(grid, x, mu=None):
    gs = _grid(grid)
    x, mu = _f64(x), _f64(mu)
    y = np.empty_like(x)
    lib().og_apply_W(C.byref(gs), _ptr(mu), _ptr(x), _ptr(y))
    return y


def apply_W_ext(grid, x, mu=None, wall_tan=None):
    """W on a field carrying Dirichlet data; wall_tan[side][component] gives the
    tangential velocity of each wall (default at rest)."""
    gs = _grid(grid)
    x, mu = _f64(x), _f64(mu)
    wt = None if wall_tan is None else _f64(np.asarray(wall_tan).reshape(18))
    y = np.empty_like(x)
    lib().og_apply_W_ext(C.byref(gs), _ptr(mu), _ptr(x), _ptr(wt), _ptr(y))
    return y


def apply_A(grid, p):
    gs = _grid(grid)
    p = _f64(p)
    m, _ = sizes(grid)
    y = np.empty(m)
    lib().og_apply_A(C.byref(gs), _ptr(p), _ptr(y))
    return y


def apply_AT(grid, x):
    gs = _grid(grid)
    x = _f64(x)
    _, n = sizes(grid)
    t = np.empty(n)
    lib().og_apply_AT(C.byref(gs), _ptr(x), _ptr(t))
    return t


def apply_M(grid, x, eta, mu=None):
    gs = _grid(grid)
    x, mu = _f64(x), _f64(mu)
    y = np.empty_like(x)
    lib().og_apply_M(C.byref(gs), _ptr(mu), float(eta), _ptr(x), _ptr(y))
    return y


def diag_M(grid, eta, mu=None):
    gs = _grid(grid)
    mu = _f64(mu)
    m, _ = sizes(grid)
    d = np.empty(m)
    lib().og_diag_M(C.byref(gs), _ptr(mu), float(eta), _ptr(d))
    return d


def pcg(grid, f, eta, mu=None, tol=1e-12, maxit=100000):
    """Jacobi-PCG on M x = f from x0 = 0.  Returns (x, status, iterations)."""
    gs = _grid(grid)
    f, mu = _f64(f), _f64(mu)
    x = np.empty_like(f)
    it = C.c_int(0)
    st = lib().og_pcg(C.byref(gs), _ptr(mu), float(eta), _ptr(f), _ptr(x),
                      float(tol), int(maxit), C.byref(it))
    return x, st, it.value


def gkb_solve(grid, g, r, eta, mu=None, tol=1e-8, delay=5, maxit=1000,
              inner_tol=1e-12, inner_maxit=100000, squared_rule=False, store_k=0,
              krylov="cg", restart=30):
    """Generalized GKB (Section 2.1) with the transformation to g = 0 and a
    Jacobi-preconditioned inner solve (krylov "cg", or "fgmres" with the given
    restart).  Returns a dict with w, p, status, K, est and the per-step
    histories (zeta, alpha, beta, est_hist, inner_iters); with store_k > 0
    also the first store_k columns of V and Q."""
    gs = _grid(grid)
    g, r, mu = _f64(g), _f64(r), _f64(mu)
    m, n = sizes(grid)
    w = np.empty(m)
    p = np.empty(n)
    zeta = np.zeros(maxit)
    alpha = np.zeros(maxit)
    beta = np.zeros(maxit)
    est_hist = np.full(maxit, -1.0)
    inner = np.zeros(maxit + 1, dtype=np.int32)
    V = np.zeros((max(store_k, 1), m))
    Q = np.zeros((max(store_k, 1), n))
    o = _GkbOpts(tol=float(tol), delay=int(delay), maxit=int(maxit),
                 inner_tol=float(inner_tol), inner_maxit=int(inner_maxit),
                 squared_rule=int(bool(squared_rule)),
                 zeta=zeta.ctypes.data, alpha=alpha.ctypes.data, beta=beta.ctypes.data,
                 est_hist=est_hist.ctypes.data, inner_iters=inner.ctypes.data,
                 store_k=int(store_k), V=V.ctypes.data, Q=Q.ctypes.data,
                 inner_krylov={"cg": 0, "fgmres": 1}[krylov], restart=int(restart))
    K = C.c_int(0)
    est = C.c_double(0.0)
    tot = C.c_int(0)
    st = lib().og_gkb_solve(C.byref(gs), _ptr(mu), float(eta), _ptr(g), _ptr(r),
                            C.byref(o), _ptr(w), _ptr(p), C.byref(K), C.byref(est),
                            C.byref(tot))
    k = K.value
    return dict(w=w, p=p, status=st, K=k, est=est.value, inner_total=tot.value,
                zeta=zeta[:k].copy(), alpha=alpha[:k].copy(), beta=beta[:k].copy(),
                est_hist=est_hist[:k].copy(), inner_iters=inner[:k + 1].copy(),
                V=V[:min(store_k, k)].copy() if store_k else None,
                Q=Q[:min(store_k, k)].copy() if store_k else None)


def gkb_fgmres(grid, g, r, eta, mu=None, tol=1e-8, restart=10, maxit=50, gkb_tol=1e-2,
               delay=2, gkb_maxit=200, inner_tol=1e-12, inner_maxit=100000, krylov="cg",
               inner_restart=30):
    """GKB as a preconditioner (Section 3): flexible GMRES on the saddle
    system, right preconditioned by one GKB run (lower-bound tolerance
    gkb_tol, delay, gkb_maxit; Jacobi-preconditioned inner solves), stopped at
    the relative residual tol.  Returns a dict with w, p, status, iterations
    (outer steps = GKB runs) and inner_total."""
    gs = _grid(grid)
    g, r, mu = _f64(g), _f64(r), _f64(mu)
    m, n = sizes(grid)
    w = np.empty(m)
    p = np.empty(n)
    o = _GkbOpts(tol=float(gkb_tol), delay=int(delay), maxit=int(gkb_maxit),
                 inner_tol=float(inner_tol), inner_maxit=int(inner_maxit), squared_rule=0,
                 store_k=0, inner_krylov={"cg": 0, "fgmres": 1}[krylov],
                 restart=int(inner_restart))
    it = C.c_int(0)
    tot = C.c_int(0)
    st = lib().og_gkb_fgmres(C.byref(gs), _ptr(mu), float(eta), _ptr(g), _ptr(r), C.byref(o),
                             float(tol), int(restart), int(maxit), _ptr(w), _ptr(p),
                             C.byref(it), C.byref(tot))
    return dict(w=w, p=p, status=st, iterations=it.value, inner_total=tot.value)


def _csr_parts(M):
    """(rowptr int32, col int32, val float64) of a scipy.sparse matrix."""
    M = M.tocsr()
    M.sort_indices()
    return (np.ascontiguousarray(M.indptr, dtype=np.int32),
            np.ascontiguousarray(M.indices, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


def csr_central_scaling(W, A):
    """Central scaling vectors (s_w, s_p) = (diag(W)^-1/2, diag(A^T diag(W)^-1
    A)^-1/2) of CSR blocks W, A (scipy.sparse)."""
    m, n = A.shape
    wp, wc, wv = _csr_parts(W)
    ap, ac, av = _csr_parts(A)
    sw, sp = np.empty(m), np.empty(n)
    st = lib().og_csr_central_scaling(m, n, _ptr(wp), _ptr(wc), _ptr(wv), _ptr(ap), _ptr(ac),
                                      _ptr(av), _ptr(sw), _ptr(sp))
    if st != OK:
        raise ValueError("central scaling needs diag(W) > 0 and no empty column of A")
    return sw, sp


def gkb_solve_csr(W, A, g, r, eta, scaling=False, tol=1e-8, delay=5, maxit=1000,
                  inner_tol=1e-12, inner_maxit=100000, krylov="cg", restart=30):
    """GKB on the assembled saddle system with CSR blocks W (m x m) and A
    (m x n) (scipy.sparse), optionally with central scaling (Section 4.1).
    Returns a dict like gkb_solve."""
    m, n = A.shape
    wp, wc, wv = _csr_parts(W)
    ap, ac, av = _csr_parts(A)
    g, r = _f64(g), _f64(r)
    w, p = np.empty(m), np.empty(n)
    zeta = np.zeros(maxit)
    inner = np.zeros(maxit + 1, dtype=np.int32)
    o = _GkbOpts(tol=float(tol), delay=int(delay), maxit=int(maxit),
                 inner_tol=float(inner_tol), inner_maxit=int(inner_maxit), squared_rule=0,
                 zeta=zeta.ctypes.data, inner_iters=inner.ctypes.data, store_k=0,
                 inner_krylov={"cg": 0, "fgmres": 1}[krylov], restart=int(restart))
    K, est, tot = C.c_int(0), C.c_double(0.0), C.c_int(0)
    st = lib().og_gkb_solve_csr(m, n, _ptr(wp), _ptr(wc), _ptr(wv), _ptr(ap), _ptr(ac),
                                _ptr(av), float(eta), int(bool(scaling)), _ptr(g), _ptr(r),
                                C.byref(o), _ptr(w), _ptr(p), C.byref(K), C.byref(est),
                                C.byref(tot))
    k = K.value
    return dict(w=w, p=p, status=st, K=k, est=est.value, inner_total=tot.value,
                zeta=zeta[:k].copy(), inner_iters=inner[:k + 1].copy())


def saddle_residual(grid, g, r, w, p, mu=None):
    """FP64 residual [g - W w - A p; r - A^T w] and its norms
    (total, velocity block, pressure block, ||[g; r]||)."""
    gs = _grid(grid)
    g, r, w, p, mu = _f64(g), _f64(r), _f64(w), _f64(p), _f64(mu)
    rw = np.empty_like(w)
    rr = np.empty_like(p)
    norms = np.zeros(4)
    lib().og_saddle_residual(C.byref(gs), _ptr(mu), _ptr(g), _ptr(r), _ptr(w), _ptr(p),
                             _ptr(rw), _ptr(rr), _ptr(norms))
    return rw, rr, norms


def dense(grid, op, eta=0.0, mu=None):
    """Dense matrix of an oracle operator ('W', 'A', 'AT', 'M') built by
    applying it to unit vectors (tiny grids only)."""
    m, n = sizes(grid)
    if op in ("W", "M", "AT"):
        cols = m
    else:
        cols = n
    out = []
    for j in range(cols):
        e = np.zeros(cols)
        e[j] = 1.0
        if op == "W":
            out.append(apply_W(grid, e, mu))
        elif op == "M":
            out.append(apply_M(grid, e, eta, mu))
        elif op == "A":
            out.append(apply_A(grid, e))
        else:
            out.append(apply_AT(grid, e))
    return np.array(out).T
