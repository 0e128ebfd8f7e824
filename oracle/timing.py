"""Wall-clock timing of the CPU oracle (test infrastructure: measures the
oracle, never used by the library).

Each run in a fresh process so that OMP_NUM_THREADS takes effect:

* Poiseuille channel 64 x 16 (eta = 1e2, tau = 1e-8, d = 5, Jacobi-PCG to
  1e-12): the complete solve, one thread and every host thread;
* 2D Stokes 512^2 (eta = 10, 8-mode forcing seed 0, pinned cell): a fixed
  sample of 200 Jacobi-PCG iterations of the first inner solve of its GKB run
  (tau_in = 1e-10), one thread and every host thread, reported as seconds per
  inner iteration (a complete oracle solve of this workload takes hours: its
  first GKB step alone needs about 1e4 inner iterations);

with the FP64 relative saddle residual of the complete solves.  Prints one
JSON line per run and a markdown table; the host is described by nproc and
the CPU model from /proc/cpuinfo.

    python oracle/timing.py
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

RUNS = {
    "poiseuille_64x16": dict(kind="poiseuille", tol=1e-8, delay=5, inner_tol=1e-12, maxit=400),
    "stokes2d_512_eta10": dict(kind="stokes2d", n=512, eta=10.0, tol=1e-9, delay=5,
                               inner_tol=1e-10, maxit=2000),
}
SAMPLE_ITERS = 200


def _child(name, sample):
    sys.path.insert(0, ROOT)
    import oracle
    import problems as P

    cfg = dict(RUNS[name])
    if cfg["kind"] == "poiseuille":
        pr = P.poiseuille_problem(64, 16, 4.0, 1e2)
    else:
        pr = P.stokes_problem(2, cfg["n"], seed=0, eta=cfg["eta"])
    oracle.lib()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0"))
    t0 = time.perf_counter()
    if sample:
        # the first inner solve, stopped after SAMPLE_ITERS iterations
        res = oracle.gkb_solve(pr.grid, pr.g, pr.r, pr.eta, mu=pr.mu, tol=cfg["tol"],
                               delay=cfg["delay"], maxit=1, inner_tol=cfg["inner_tol"],
                               inner_maxit=SAMPLE_ITERS)
        dt = time.perf_counter() - t0
        print(json.dumps(dict(run=name, threads=threads, sample_iterations=SAMPLE_ITERS,
                              seconds=round(dt, 3),
                              seconds_per_iteration=dt / SAMPLE_ITERS)), flush=True)
        return
    res = oracle.gkb_solve(pr.grid, pr.g, pr.r, pr.eta, mu=pr.mu, tol=cfg["tol"],
                           delay=cfg["delay"], maxit=cfg["maxit"], inner_tol=cfg["inner_tol"],
                           inner_maxit=10 ** 8)
    dt = time.perf_counter() - t0
    _, _, nr = oracle.saddle_residual(pr.grid, pr.g, pr.r, res["w"], res["p"], mu=pr.mu)
    print(json.dumps(dict(run=name, threads=threads, seconds=round(dt, 3),
                          status=res["status"], K=res["K"], inner_iterations=res["inner_total"],
                          residual=nr[0] / nr[3])), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "--child":
        _child(sys.argv[2], sys.argv[3] == "1")
        return
    nproc = os.cpu_count() or 1
    plan = [("poiseuille_64x16", 1, 0), ("poiseuille_64x16", nproc, 0),
            ("stokes2d_512_eta10", 1, 1), ("stokes2d_512_eta10", nproc, 1)]
    print(f"# host: nproc {nproc}, {_cpu_model()}", flush=True)
    rows = []
    for name, threads, sample in plan:
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--child", name,
                              str(sample)], env=env, capture_output=True, text=True, check=True)
        line = out.stdout.strip().splitlines()[-1]
        print(line, flush=True)
        rows.append(json.loads(line))
    print("\n| run | threads | what | s | result |")
    print("|---|---|---|---|---|")
    for r in rows:
        if "sample_iterations" in r:
            print(f"| {r['run']} | {r['threads']} | {r['sample_iterations']} inner iterations "
                  f"| {r['seconds']} | {r['seconds_per_iteration']:.4f} s per iteration |")
        else:
            print(f"| {r['run']} | {r['threads']} | complete solve (status {r['status']}, K "
                  f"{r['K']}, {r['inner_iterations']} inner iterations) | {r['seconds']} | "
                  f"FP64 residual {r['residual']:.2e} |")


if __name__ == "__main__":
    main()
