"""MI355X-native generalized Golub-Kahan bidiagonalization (GKB) solver for
MAC-discretized Stokes saddle-point systems.

Thin Python binding over the C-ABI of ``libgkb.so`` (``include/gkb.h``):
arguments are marshalled here, every step of the solve runs in HIP kernels.
PyTorch is used only for device memory and streams.

    s = Solver(grid, mu=None, eta=1e3, inner="mg", precision="fp64")
    w, p, info = s.solve(g, r, tol=1e-8, delay=5)   # g, r: cuda float64 tensors
"""
from __future__ import annotations

import ctypes as C

from . import _abi

__all__ = ["Solver", "CsrSolver", "library", "CNN", "residual_noalloc"]


def library():
    """The loaded C library (raises if it has not been built)."""
    return _abi.lib()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _grid_struct(grid):
    gs = _abi.Grid()
    gs.dim = int(grid.dim)
    for a in range(3):
        gs.n[a] = int(grid.n[a]) if a < grid.dim else 1
    gs.h = float(grid.h)
    for s in range(6):
        gs.bc[s] = int(grid.bc[s])
    gs.pin_cell = int(grid.pin)
    return gs


def residual_noalloc(grid, g, r, w, p, res_w=None, res_r=None):
    """FP64 saddle residual for mu = 1 without a solver context and without
    device allocation by the library (gkb_residual_noalloc).  g, w (faces) and
    r, p (cells): contiguous cuda float64 tensors; res_r (cells) is required by
    the C call and created here when not given.  Returns (norms, res_w, res_r)
    with norms = (||res||, ||res_w||, ||res_r||, ||[g; r]||)."""
    import torch
    for t in (g, r, w, p, res_w, res_r):
        if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("expected contiguous cuda float64 tensors")
    if res_r is None:
        res_r = torch.empty_like(r)
    norms = (C.c_double * 4)()
    gs = _grid_struct(grid)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _abi.check(_abi.lib().gkb_residual_noalloc(C.byref(gs), _ptr(g), _ptr(r), _ptr(w), _ptr(p),
                                               _ptr(res_w), _ptr(res_r), norms, stream),
               "gkb_residual_noalloc")
    return list(norms), res_w, res_r


class Solver:
    """One solver context (``gkb_setup``) for a grid, viscosity and eta.

    grid: object with ``dim``, ``n`` (3 ints), ``h``, ``bc`` (6 ints), ``pin``.
    mu: host array of cell viscosities (numpy / CPU tensor) or None (mu = 1).
    eta: augmented-Lagrangian parameter (the paper's nu; 0 = off).
    options: precision ("fp64" | "mixed"), inner ("jacobi" | "mg" | "learned"),
      smoother ("jacobi" | "hybrid"), krylov ("cg" | "fgmres"), fgmres_restart,
      method ("solver" | "precond": GKB as the solver or as the preconditioner
      of an outer FGMRES), outer_restart, cnn_weights (checkpoint path loaded at
      setup), learned_min_gain, mg_transfer ("auto" | "div" | "smooth"),
      mg_levels, nu_pre, nu_post, inner_tol,
      inner_maxit, maxit, refine_tol, max_sweeps, check_every, use_graphs,
      stencil, max_workspace_bytes.
    """

    def __init__(self, grid, mu=None, eta=0.0, **options):
        import numpy as np

        L = _abi.lib()
        self.grid = grid
        self.eta = float(eta)
        opt = self._options(options)
        self._mu = None
        mu_ptr = None
        if mu is not None:
            self._mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
            mu_ptr = self._mu.ctypes.data_as(C.c_void_p)
        ctx = C.c_void_p()
        gs = _grid_struct(grid)
        _abi.check(L.gkb_setup(C.byref(gs), mu_ptr, self.eta, C.byref(opt), C.byref(ctx)),
                   "gkb_setup")
        self._finish(ctx)

    def _options(self, options, defaults=None):
        import torch

        L = _abi.lib()
        opt = _abi.Options()
        L.gkb_default_options(C.byref(opt))
        for k, v in dict(defaults or {}, **options).items():
            if k == "precision":
                v = {"fp64": _abi.FP64, "mixed": _abi.MIXED}.get(v, v)
            elif k == "inner":
                v = _abi.INNER.get(v, v)
            elif k == "smoother":
                v = _abi.SMOOTHERS.get(v, v)
            elif k == "krylov":
                v = _abi.KRYLOV.get(v, v)
            elif k == "method":
                v = _abi.METHODS.get(v, v)
            elif k == "mg_transfer":
                v = _abi.TRANSFERS.get(v, v)
            elif k == "cnn_weights":
                v = None if v is None else str(v).encode()
            if not hasattr(opt, k):
                raise TypeError(f"unknown option {k}")
            setattr(opt, k, v)
        self.options = {f: getattr(opt, f) for f, _ in _abi.Options._fields_}
        self._weights_path = opt.cnn_weights  # kept alive through gkb_setup
        opt.hip_stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return opt

    def _finish(self, ctx):
        import torch

        L = _abi.lib()
        self._ctx = ctx
        m_full, n_cells, mu_n, nu_n = (C.c_long() for _ in range(4))
        L.gkb_sizes(ctx, C.byref(m_full), C.byref(n_cells), C.byref(mu_n), C.byref(nu_n))
        self.m_full, self.n_cells = m_full.value, n_cells.value
        self.m_unknown, self.n_unknown = mu_n.value, nu_n.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    # ---------------------------------------------------------------- helpers
    def _vec(self, t, n, dtype=None):
        import torch
        dtype = dtype or torch.float64
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"expected a contiguous cuda {dtype} tensor of {n} entries")
        return t

    def _new(self, n, dtype=None):
        import torch
        return torch.empty(n, dtype=dtype or torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_ctx", None):
            _abi.lib().gkb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- solving
    def solve(self, g, r, tol=1e-8, delay=5, w=None, p=None):
        """gkb_solve: returns (w, p, info) with info = status, iterations,
        error_estimate and the statistics of the solve."""
        L = _abi.lib()
        g = self._vec(g, self.m_full)
        r = self._vec(r, self.n_cells)
        w = self._new(self.m_full) if w is None else self._vec(w, self.m_full)
        p = self._new(self.n_cells) if p is None else self._vec(p, self.n_cells)
        K = C.c_int(0)
        est = C.c_double(0.0)
        rc = L.gkb_solve(self._ctx, _ptr(g), _ptr(r), float(tol), int(delay), _ptr(w), _ptr(p),
                         C.byref(K), C.byref(est))
        _abi.check(rc, "gkb_solve")
        info = dict(status=rc, iterations=K.value, error_estimate=est.value)
        info.update(self.stats())
        return w, p, info

    def stats(self):
        st = _abi.Stats()
        _abi.check(_abi.lib().gkb_stats(self._ctx, C.byref(st)), "gkb_stats")
        n = st.history_len
        return dict(sweeps=st.sweeps, outer_iterations=st.outer_iterations,
                    inner_iterations=st.inner_iterations, inner_solves=st.inner_solves,
                    fallbacks=st.fallbacks, learned_solves=st.learned_solves,
                    residual=st.residual,
                    seconds_solve=st.seconds_solve, zeta=list(st.zeta[:n]),
                    estimate=list(st.estimate[:n]), workspace_bytes=st.workspace_bytes,
                    mg_levels=st.mg_levels, omega=list(st.omega[:st.mg_levels]),
                    omega_edge=list(st.omega_edge[:st.mg_levels]),
                    learned_gain=st.learned_gain,
                    learned_fallback_reason=st.learned_fallback_reason,
                    learned_fallback_iteration=st.learned_fallback_iteration,
                    outer_krylov_iterations=st.outer_krylov_iterations,
                    mg_transfer={1: "div", 2: "smooth"}.get(st.mg_transfer, "none"))

    def apply(self, op, x, precision="fp64"):
        """y = op(x) for op in W, A, AT, M, diag (gkb_apply)."""
        import torch
        prec = _abi.FP64 if precision == "fp64" else _abi.MIXED
        dt = torch.float64 if prec == _abi.FP64 else torch.float32
        n_in = self.n_cells if op == "A" else self.m_full
        n_out = self.n_cells if op == "AT" else self.m_full
        if op != "diag":
            self._vec(x, n_in, dt)
        y = self._new(n_out, dt)
        _abi.check(_abi.lib().gkb_apply(self._ctx, _abi.OPS[op], prec,
                                        None if op == "diag" else _ptr(x), _ptr(y)), "gkb_apply")
        return y

    def precondition(self, r, precision="fp64"):
        import torch
        prec = _abi.FP64 if precision == "fp64" else _abi.MIXED
        dt = torch.float64 if prec == _abi.FP64 else torch.float32
        self._vec(r, self.m_full, dt)
        z = self._new(self.m_full, dt)
        _abi.check(_abi.lib().gkb_precondition(self._ctx, prec, _ptr(r), _ptr(z)),
                   "gkb_precondition")
        return z

    def inner_solve(self, f, tol=0.0):
        self._vec(f, self.m_full)
        x = self._new(self.m_full)
        it = C.c_int(0)
        rc = _abi.lib().gkb_inner_solve(self._ctx, _ptr(f), _ptr(x), float(tol), C.byref(it))
        _abi.check(rc, "gkb_inner_solve")
        return x, it.value

    def time_kernel(self, kernel="smooth", reps=50):
        """Average duration (ms) of one finest-grid inner kernel, timed with HIP
        events on the library's stream (gkb_time_kernel)."""
        ms = C.c_double(0.0)
        _abi.check(_abi.lib().gkb_time_kernel(self._ctx, _abi.KERNELS[kernel], int(reps),
                                              C.byref(ms)), "gkb_time_kernel")
        return ms.value

    def attach_cnn(self, net):
        """Use a CNN (paper_2001_10424_amd.CNN, or a checkpoint path) in the
        learned inner solves."""
        from .cnn import CNN, attach
        if isinstance(net, str):
            net = CNN.load(net)
        attach(self, net)
        return net

    def residual(self, g, r, w, p, want_vectors=False):
        """FP64 saddle residual (gkb_residual): returns (norms, res_w, res_r);
        norms = (||res||, ||res_w||, ||res_r||, ||[g; r]||)."""
        norms = (C.c_double * 4)()
        rw = self._new(self.m_full) if want_vectors else None
        rr = self._new(self.n_cells) if want_vectors else None
        _abi.check(_abi.lib().gkb_residual(self._ctx, _ptr(g), _ptr(r), _ptr(w), _ptr(p),
                                           _ptr(rw), _ptr(rr), norms), "gkb_residual")
        return list(norms), rw, rr


class CsrSolver(Solver):
    """A solver context for an assembled saddle system (gkb_setup_csr).

    W: m x m and A: m x n scipy.sparse matrices (any format; converted to
    CSR with int32 indices), eta as for Solver, scaling "central" (the
    block scaling blockdiag(D^-1/2, R^-1/2) of Section 4.1) or "none".  The
    inner solver is Jacobi-preconditioned CG (krylov="cg") or FGMRES.
    solve(g, r) takes and returns cuda float64 tensors of lengths m and n."""

    def __init__(self, W, A, eta=0.0, scaling="central", **options):
        import numpy as np

        L = _abi.lib()
        self.grid = None
        self.eta = float(eta)
        m, n = A.shape
        if W.shape != (m, m):
            raise ValueError("W must be m x m and A m x n")
        opt = self._options(options, defaults=dict(inner="jacobi"))
        keep = []
        sysd = _abi.Csr()
        sysd.m, sysd.n = int(m), int(n)
        for name, M in (("w", W), ("a", A)):
            M = M.tocsr()
            M.sort_indices()
            ptr = np.ascontiguousarray(M.indptr, dtype=np.int32)
            col = np.ascontiguousarray(M.indices, dtype=np.int32)
            val = np.ascontiguousarray(M.data, dtype=np.float64)
            keep += [ptr, col, val]
            setattr(sysd, name + "_rowptr", ptr.ctypes.data_as(C.POINTER(C.c_int)))
            setattr(sysd, name + "_col", col.ctypes.data_as(C.POINTER(C.c_int)))
            setattr(sysd, name + "_val", val.ctypes.data_as(C.POINTER(C.c_double)))
        mode = {"none": _abi.SCALE_NONE, "central": _abi.SCALE_CENTRAL}[scaling]
        ctx = C.c_void_p()
        _abi.check(L.gkb_setup_csr(C.byref(sysd), self.eta, mode, C.byref(opt), C.byref(ctx)),
                   "gkb_setup_csr")
        del keep
        self._finish(ctx)


from .cnn import CNN  # noqa: E402
