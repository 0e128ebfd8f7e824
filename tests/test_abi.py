"""The C-ABI without a GPU: the built library loads, exports every function
that include/gkb.h and include/gkb_cnn.h declare, and its host-only paths
(default options, error strings, argument validation that fails before any
HIP call) behave as the headers state.  No compute call is made here."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gkb.h", "gkb_cnn.h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # drop comments
        text = re.sub(r"#[^\n]*", " ", text)                  # and preprocessor lines
        for m in re.finditer(r"\b(gkb_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2001_10424_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libgkb.so is not built (python __graft_entry__.py build)")
    return _abi.lib()


def test_headers_declare_the_entry_points():
    names = _declared()
    for n in ("gkb_setup", "gkb_solve", "gkb_stats", "gkb_destroy", "gkb_default_options",
              "gkb_strerror", "gkb_cnn_create", "gkb_cnn_train", "gkb_attach_cnn"):
        assert n in names
    assert len(names) >= 25, names


def test_library_exports_every_declared_function(lib):
    from paper_2001_10424_amd import _abi
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                             text=True, check=True).stdout
        exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
        assert not [n for n in _declared() if n not in exported]


def test_default_options(lib):
    from paper_2001_10424_amd import _abi
    o = _abi.Options()
    lib.gkb_default_options(C.byref(o))
    assert (o.precision, o.inner, o.mg_levels, o.nu_pre, o.nu_post) == (0, 1, 0, 2, 2)
    assert o.inner_tol == 1e-10 and o.inner_maxit == 10000 and o.maxit == 500
    assert o.refine_tol == 0.0 and o.max_sweeps == 10 and o.check_every == 8
    assert o.use_graphs == 1 and o.stencil == 0 and o.smoother == 0
    assert o.hip_stream is None and o.max_workspace_bytes == 0
    assert (o.krylov, o.fgmres_restart, o.method, o.outer_restart) == (0, 30, 0, 10)
    assert o.cnn_weights is None and o.learned_min_gain == 0.05
    assert o.mg_transfer == 0  # GKB_TRANSFER_AUTO


def test_error_strings(lib):
    expect = {0: "ok", 1: "maximum", -1: "invalid", -2: "memory", -3: "HIP", -4: "non-finite",
              -5: "inner", 7: "unknown"}
    for code, word in expect.items():
        assert word in lib.gkb_strerror(code).decode()


def _grid(dim=3, n=(8, 8, 8), h=0.125, bc=(0,) * 6, pin=0):
    from paper_2001_10424_amd import _abi
    g = _abi.Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a]
    g.h = h
    for s in range(6):
        g.bc[s] = bc[s]
    g.pin_cell = pin
    return g


def test_setup_rejects_invalid_arguments_before_any_device_work(lib):
    from paper_2001_10424_amd import _abi
    ctx = C.c_void_p()
    bad = [
        (_grid(dim=4), 1.0),                    # dimension
        (_grid(n=(1, 8, 8)), 1.0),              # fewer than 2 cells
        (_grid(h=0.0), 1.0),                    # cell size
        (_grid(), -1.0),                        # negative eta
        (_grid(bc=(2, 0, 0, 0, 0, 0)), 1.0),    # unknown boundary type
        (_grid(pin=512), 1.0),                  # pinned cell out of range
        (_grid(bc=(1,) * 6, pin=-1), 0.0),      # every side natural
    ]
    for g, eta in bad:
        assert lib.gkb_setup(C.byref(g), None, eta, None, C.byref(ctx)) == _abi.GKB_EINVAL
        assert not ctx.value
    o = _abi.Options()
    lib.gkb_default_options(C.byref(o))
    for field, value in (("precision", 5), ("inner", 9), ("nu_pre", -1), ("maxit", 0),
                         ("check_every", 0), ("stencil", 3), ("smoother", 4), ("krylov", 2),
                         ("fgmres_restart", 0), ("fgmres_restart", 65), ("method", 2),
                         ("method", 1),  # GKB as preconditioner needs refine_tol > 0
                         ("outer_restart", 0), ("outer_restart", 33),
                         ("learned_min_gain", float("nan")),
                         ("mg_transfer", -1), ("mg_transfer", 3)):
        oo = _abi.Options()
        C.memmove(C.byref(oo), C.byref(o), C.sizeof(o))
        setattr(oo, field, value)
        assert lib.gkb_setup(C.byref(_grid()), None, 1.0, C.byref(oo), C.byref(ctx)) == \
            _abi.GKB_EINVAL, field
    oo = _abi.Options()
    C.memmove(C.byref(oo), C.byref(o), C.sizeof(o))
    oo.cnn_weights = b"/nonexistent/net.bin"  # network weights need the learned inner solver
    assert lib.gkb_setup(C.byref(_grid()), None, 1.0, C.byref(oo), C.byref(ctx)) == _abi.GKB_EINVAL
    mu = (C.c_double * 512)(*([1.0] * 511 + [-1.0]))  # non-positive viscosity
    assert lib.gkb_setup(C.byref(_grid()), mu, 1.0, None, C.byref(ctx)) == _abi.GKB_EINVAL
    assert lib.gkb_setup(C.byref(_grid()), None, 1.0, None, None) == _abi.GKB_EINVAL


def test_null_context_calls_fail_cleanly(lib):
    from paper_2001_10424_amd import _abi
    st = _abi.Stats()
    assert lib.gkb_stats(None, C.byref(st)) == _abi.GKB_EINVAL
    assert lib.gkb_solve(None, None, None, 1e-8, 5, None, None, None, None) == _abi.GKB_EINVAL
    # the allocation-free residual validates its grid before any device work
    g = _grid(h=-1.0)
    norms = (C.c_double * 4)()
    one = C.c_void_p(8)  # never dereferenced: the grid is rejected first
    assert lib.gkb_residual_noalloc(C.byref(g), one, one, one, one, None, one, norms,
                                    None) == _abi.GKB_EINVAL
    assert lib.gkb_residual_noalloc(None, one, one, one, one, None, one, norms,
                                    None) == _abi.GKB_EINVAL
    lib.gkb_destroy(None)
    ms = C.c_double()
    for k in (0, 3, 4, 5, -1):
        assert lib.gkb_time_kernel(None, k, 10, C.byref(ms)) == _abi.GKB_EINVAL
    bad = C.c_void_p()
    ch = (C.c_int * 3)(4, 40, 3)  # a layer wider than 16 channels
    assert lib.gkb_cnn_create(3, 2, ch, 0, C.byref(bad)) == _abi.GKB_EINVAL
    assert lib.gkb_cnn_load(b"/nonexistent/weights.bin", C.byref(bad)) == _abi.GKB_EINVAL
