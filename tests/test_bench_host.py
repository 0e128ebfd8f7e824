"""Host-side pieces of bench.py (CPU): the one-GPU guard, the timed-mode
table, the roofline byte count of the dominant kernel and the counter
summary it reads."""
import os
import subprocess
import sys

import pytest

import bench
import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_timed_modes_share_one_stopping_protocol():
    """Every defect-correction mode stops each sweep on the same loose
    lower-bound tolerance with delay 2; fp64_gkb1 is the single GKB run of
    the paper (tau 1e-9, delay 5); V(2,2) Jacobi or V(1,1) hybrid."""
    for name, (prec, inner, tol, itol, delay, smoother, nu) in bench.MODES.items():
        assert prec in ("fp64", "mixed") and inner in ("mg", "learned"), name
        assert (smoother, nu) in (("jacobi", 2), ("hybrid", 1)), name
        assert 0 < itol < 1e-2, name
        if name == "fp64_gkb1":
            assert (tol, delay) == (1e-9, 5)
        elif name == "fp64_gkb_precond":
            assert delay == 2 and tol < 0.1  # one preconditioning GKB run per step
        else:
            assert (tol, delay) == (0.3, 2), name
    assert bench.MODES["mixed_learned"][:1] == ("mixed",)
    assert set(bench.EXTRA) <= set(bench.MODES)


def test_roofline_bytes_of_the_prolongation_sweep():
    """x, b read and y written on the 128^3 full-face layout plus the coarse
    correction read on the 64^3 one, 4 B each: the figure the bench divides
    by the measured launch time."""
    pr = P.stokes_problem(3, 8, seed=0, eta=1e3, lid=True)  # grid object only
    g = P.Grid(3, (128, 128, 128), 1 / 128, pr.grid.bc, pr.grid.pin)
    m_full = sum((128 + (c == 0)) * (128 + (c == 1)) * (128 + (c == 2)) for c in range(3))
    assert m_full == 6340608
    assert bench.coarse_faces(g) == 3 * 65 * 64 * 64 == 798720
    assert (3 * m_full + bench.coarse_faces(g)) * 4 == 79282176


def test_counter_summary_matches_the_kernel_sources():
    """The committed counter summary names the hash of the stencil sources it
    was taken on; while it matches, the bench reports its traffic."""
    traffic = bench.counter_traffic()
    if traffic is None:
        pytest.skip("stencil sources changed since the counters were taken")
    assert 79282176 <= traffic <= 1.2 * 79282176
