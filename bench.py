"""Benchmark: time to the periodic adjoint gradient on one MI355X.

One step = the whole hot path of the method on the flapping-cylinder
workload (32x96 O-grid, DG p=3, 40x40 Jacobian blocks, DIRK3 with 100 steps
per period): from the free stream, Newton-Krylov shooting to
||u^(Nt) - u0||_2 <= 1e-8 (primal sweeps with per-stage Newton and
block-Jacobi GMRES(30) at 1e-10, tangent sweeps as matvecs), then the
periodic adjoint (Alg. 3) and the gradient of both time-averaged QoIs with
respect to mu = (h0, theta0, phi).  Inputs (mesh tables, GCL field, initial
state) are resident in HBM before the timed region.

Prints one JSON line.  --gpus N > 1 is refused: the build targets one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1512_00616_amd import inputs  # noqa: E402

HBM_PEAK_GBS = 8000.0


def spmv_bytes(Nr, Nth, p):
    """Algorithmic bytes of one stage-operator apply y = (M - c J) x:
    every nonzero block once (diagonal + two per interior face), x and y once."""
    np_ = (p + 1) * (p + 2) // 2
    b = 4 * np_
    Ne = 2 * Nr * Nth
    n_int_faces = 3 * Ne // 2 - Nth          # wall and far-field edges are unpaired
    nblocks = Ne + 2 * n_int_faces
    Nu = Ne * b
    return nblocks * b * b * 8 + 2 * Nu * 8


def cpu_baseline(work, counts, mu, budget_s=30.0):
    """Oracle timed on the host cores on a bounded sample of the same
    workload: one residual, one Jacobian assembly and one block-Jacobi GMRES
    stage solve at the benchmark's discretisation; the time to gradient is
    composed from these unit times and the GPU run's own counts."""
    from oracle.oracle import Oracle
    nthreads = os.cpu_count() or 1
    o = Oracle(lin_solver=1, lin_rtol=1e-10, nthreads=nthreads, **work)
    o.set_params(mu)
    u = o.freestream()
    t0 = time.perf_counter()
    o.residual(1, 1, u)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    J = o.jacobian(1, 1, u)
    t_jac = time.perf_counter() - t0
    rhs = o.mass(inputs.random_vectors(o.Nu, 1, seed=7)[0])
    c = (1.0 / work["Nt"]) * 0.4358665215084590
    _, lin0 = o.counters()
    t0 = time.perf_counter()
    o.stage_solve(J, c, rhs)
    t_sol = time.perf_counter() - t0
    _, lin1 = o.counters()
    its = max(lin1 - lin0, 1)
    t_it = t_sol / its
    est = (counts["residuals"] * t_res + counts["jacobians"] * t_jac + counts["gmres_its"] * t_it)
    return {
        "value": est, "unit": "s", "cores": nthreads, "kind": "oracle",
        "sample": ("one residual (%.3fs), one complex-step Jacobian (%.2fs) and one GMRES stage solve "
                   "(%d its, %.4fs/it) at the benchmark discretisation; composed with the GPU run's "
                   "counts (%d residuals, %d Jacobians, %d GMRES its)"
                   % (t_res, t_jac, its, t_it, counts["residuals"], counts["jacobians"], counts["gmres_its"])),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="circle-32x96-p3-nt100", choices=sorted(inputs.WORKLOADS))
    ap.add_argument("--shoot-tol", type=float, default=1e-8)
    ap.add_argument("--shoot-eta", type=float, default=1e-3)
    ap.add_argument("--adj-rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method's sweeps are sequential in time and this build "
              "measures one MI355X; multi-GPU runs are not supported", file=sys.stderr)
        return 2

    from paper_1512_00616_amd import pa

    work = inputs.WORKLOADS[args.workload]
    mu = np.array(inputs.MU_NOMINAL)
    t_setup = time.perf_counter()
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, **work, **inputs.PHYSICS)
    s.set_params(mu)
    setup_s = time.perf_counter() - t_setup

    def step():
        s.set_freestream()
        rep = s.shoot(tol=args.shoot_tol, eta=args.shoot_eta, maxit=40)
        q, dJ, arep = s.adjoint_gradient(rtol=args.adj_rtol)
        return rep, q, dJ, arep

    for _ in range(args.warmup):
        step()
    s.set_timing(True)
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        reps.append(step())
    t1 = time.perf_counter()
    ms_spmv, n_spmv = s.kernel_time(pa.PA_K_SPMV)
    ms_pre, n_pre = s.kernel_time(pa.PA_K_PRECOND)
    ms_jac, n_jac = s.kernel_time(pa.PA_K_JACOBIAN)
    ms_res, n_res = s.kernel_time(pa.PA_K_RESIDUAL)
    s.set_timing(False)
    step_s = (t1 - t0) / args.steps
    rep, q, dJ, arep = reps[-1]
    gmres_its = rep.stage_gmres_its + arep.stage_gmres_its
    # stage solves: primal Newton corrections + tangent/adjoint stage solves
    nst = 3 * work["Nt"]
    sweeps_lin = rep.krylov_its + arep.sweeps
    stage_solves = rep.stage_newton_its + nst * sweeps_lin
    Nu = s.Nu
    bytes_spmv = spmv_bytes(work["Nr"], work["Nth"], work["p"])
    avg_spmv_s = ms_spmv / max(n_spmv, 1) / 1e3
    achieved = bytes_spmv / avg_spmv_s / 1e9
    out = {
        "metric": "time-to-periodic-adjoint-gradient (s) at 1e-8 periodicity",
        "value": step_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, **work, "mu": list(mu), "shoot_tol": args.shoot_tol,
                   "shoot_eta": args.shoot_eta, "adj_rtol": args.adj_rtol, "stage_gmres": "block-Jacobi GMRES(30) 1e-10"},
        "stage_solve_dof_per_s": stage_solves * Nu / step_s,
        "hbm_gbs_spmv": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_bsr_apply<10>",
                     "bytes_per_launch": bytes_spmv, "avg_launch_us": avg_spmv_s * 1e6, "launches": n_spmv},
        "kernels_ms": {"spmv": ms_spmv, "precond": ms_pre, "jacobian": ms_jac, "residual": ms_res},
        "counts": {"newton": rep.newton_its, "tangent_sweeps": rep.krylov_its, "primal_sweeps": rep.primal_sweeps,
                   "stage_newton": rep.stage_newton_its, "stage_gmres": gmres_its,
                   "adjoint_krylov": list(arep.krylov_its), "adjoint_sweeps": arep.sweeps},
        "periodicity": {"res0": rep.res0, "res": rep.res},
        "qoi": list(q), "dJdmu": dJ.tolist(),
        "setup_s": setup_s,
        "device_gb": s.device_bytes / 1e9,
    }
    if not args.no_cpu_baseline:
        counts = {"residuals": n_res // max(args.steps, 1), "jacobians": n_jac // max(args.steps, 1),
                  "gmres_its": gmres_its}
        try:
            out["cpu_baseline"] = cpu_baseline(work, counts, mu)
        except Exception as e:  # the oracle is optional on the box: report, do not fail the bench
            out["cpu_baseline"] = {"value": None, "error": str(e)}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
