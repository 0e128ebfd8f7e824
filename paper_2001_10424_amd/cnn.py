"""Binding of the learned preconditioner network (include/gkb_cnn.h):
argument marshalling only, every forward / backward / optimiser step runs in
the HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class CNN:
    """Convolutional preconditioner network (gkb_cnn_*).

    dim: 2 or 3; channels: (c_0, ..., c_L), each <= 16."""

    def __init__(self, dim=3, channels=(4, 8, 8, 3), seed=0, _handle=None):
        L = _abi.lib()
        self.dim = dim
        self.channels = tuple(channels)
        if _handle is not None:
            self._h = _handle
        else:
            ch = (C.c_int * len(channels))(*channels)
            h = C.c_void_p()
            _abi.check(L.gkb_cnn_create(dim, len(channels) - 1, ch, int(seed), C.byref(h)),
                       "gkb_cnn_create")
            self._h = h
        self.n_params = L.gkb_cnn_param_count(self._h)

    @classmethod
    def load(cls, path, dim=None, channels=None):
        h = C.c_void_p()
        _abi.check(_abi.lib().gkb_cnn_load(path.encode(), C.byref(h)), "gkb_cnn_load")
        obj = cls.__new__(cls)
        obj._h = h
        obj.n_params = _abi.lib().gkb_cnn_param_count(h)
        obj.dim = dim
        obj.channels = channels
        return obj

    def save(self, path):
        _abi.check(_abi.lib().gkb_cnn_save(self._h, path.encode()), "gkb_cnn_save")

    def close(self):
        if getattr(self, "_h", None):
            _abi.lib().gkb_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        _abi.check(_abi.lib().gkb_cnn_get_params(self._h, out.ctypes.data_as(C.c_void_p)),
                   "gkb_cnn_get_params")
        return out

    @params.setter
    def params(self, values):
        v = np.ascontiguousarray(np.asarray(values, dtype=np.float32))
        assert v.size == self.n_params
        _abi.check(_abi.lib().gkb_cnn_set_params(self._h, v.ctypes.data_as(C.c_void_p)),
                   "gkb_cnn_set_params")

    @staticmethod
    def _geom(x, dim):
        # x: [batch, (nz,) ny, nx, c]
        if dim == 2:
            b, ny, nx = x.shape[:3]
            return nx, ny, 1, b
        b, nz, ny, nx = x.shape[:4]
        return nx, ny, nz, b

    def forward(self, x):
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        nx, ny, nz, b = self._geom(x, self.dim)
        y = torch.empty(x.shape[:-1] + (self.channels[-1],), dtype=torch.float32, device=x.device)
        _abi.check(_abi.lib().gkb_cnn_forward(self._h, nx, ny, nz, b, _p(x), _p(y)),
                   "gkb_cnn_forward")
        return y

    def backward(self, x, dy, want_dx=True):
        import torch
        nx, ny, nz, b = self._geom(x, self.dim)
        dx = torch.empty_like(x) if want_dx else None
        g = np.empty(self.n_params, dtype=np.float32)
        _abi.check(_abi.lib().gkb_cnn_backward(self._h, nx, ny, nz, b, _p(x), _p(dy.contiguous()),
                                               _p(dx), g.ctypes.data_as(C.c_void_p)),
                   "gkb_cnn_backward")
        return g, dx

    def adam_step(self, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        gp = None
        if grad is not None:
            grad = np.ascontiguousarray(np.asarray(grad, dtype=np.float32))
            gp = grad.ctypes.data_as(C.c_void_p)
        _abi.check(_abi.lib().gkb_cnn_adam_step(self._h, gp, lr, beta1, beta2, eps),
                   "gkb_cnn_adam_step")

    def train(self, inputs, targets, grid_n, crop=32, batch=8, steps=500, lr=2e-3, seed=0):
        """gkb_cnn_train on stored pairs inputs [pairs, cells, c_0],
        targets [pairs, cells, c_L] of grids with grid_n = (nx, ny, nz) cells.
        Returns the loss of every step."""
        nx, ny, nz = grid_n
        losses = np.zeros(steps, dtype=np.float32)
        _abi.check(_abi.lib().gkb_cnn_train(self._h, _p(inputs), _p(targets), inputs.shape[0],
                                            nx, ny, nz, crop, batch, steps, float(lr), int(seed),
                                            losses.ctypes.data_as(C.c_void_p)), "gkb_cnn_train")
        return losses

    def evaluate(self, inputs, targets, grid_n):
        nx, ny, nz = grid_n
        out = C.c_double(0.0)
        _abi.check(_abi.lib().gkb_cnn_eval(self._h, _p(inputs), _p(targets), inputs.shape[0], nx,
                                           ny, nz, C.byref(out)), "gkb_cnn_eval")
        return out.value


def attach(solver, net):
    """Use `net` in the solver's learned inner solves (gkb_attach_cnn)."""
    _abi.check(_abi.lib().gkb_attach_cnn(solver._ctx, None if net is None else net._h),
               "gkb_attach_cnn")
    solver._cnn = net


def capture_pairs(solver, g, r, tol, max_pairs, iters=(0, 2, 5, 10), delay=5):
    """Run one gkb_solve with pair capture on; returns (inputs, targets) device
    tensors of the captured pairs (gkb_set_capture)."""
    import torch
    G = solver.grid
    cells = solver.n_cells
    dim = G.dim
    inp = torch.zeros((max_pairs, cells, dim + 1), dtype=torch.float32, device=solver.device)
    tgt = torch.zeros((max_pairs, cells, dim), dtype=torch.float32, device=solver.device)
    it = (C.c_int * len(iters))(*iters)
    L = _abi.lib()
    _abi.check(L.gkb_set_capture(solver._ctx, _p(inp), _p(tgt), max_pairs, len(iters), it),
               "gkb_set_capture")
    try:
        solver.solve(g, r, tol=tol, delay=delay)
        n = C.c_int(0)
        L.gkb_capture_count(solver._ctx, C.byref(n))
    finally:
        L.gkb_set_capture(solver._ctx, None, None, 0, 0, None)
    return inp[:n.value], tgt[:n.value]
