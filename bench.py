"""Benchmark of the periodic-adjoint hot path on one MI355X.

Workload: flapping cylinder, 32x96 O-grid, DG p=3 (40x40 Jacobian blocks,
245,760 DOFs), DIRK3 with 100 steps per period, heave/pitch mu = (0.25,
10 deg, pi/2), from the free stream.  One step runs every part of the path at
that size:
  * Newton-Krylov shooting step (Alg. 2): primal period with per-stage Newton
    and block-Jacobi GMRES(30) at 1e-10, a matrix-free Krylov solve of
    (Phi - I) Delta = R with tangent sweeps as matvecs (basis capped at K),
    and the line-searched update u0 - lam Delta (each trial is a primal period);
  * periodic adjoint (Alg. 3) for both QoIs (forced backward sweeps,
    adjoint-sensitivity sweeps as matvecs, basis capped at K) and the
    gradient dJ/dmu (eq. funcl-grad-nosens-dirk).
Every stage solve inside the step is converged to 1e-10; the reported value is
the stage-solve throughput (DOFs x stage solves per second).

A step takes tens of seconds, so --steps and --warmup are upper bounds: the
timed steps stop when the next one would end past --budget-s (default 100 s;
at least one step is timed) and the warm-up steps likewise within
--warmup-budget-s.  The JSON line reports the steps actually run.

The roofline object names the stage-operator apply with the largest total
time over the timed steps (HIP events on the library stream that every 8th
launch records at its kernel's start and end); the other applies and the
stage-GMRES vector kernels are
reported beside it.  The oracle is timed on the host on a bounded sample
(one residual, one Jacobian, one stage solve at the same size) and composed
with the step's counts.

On this mesh the T-periodic orbit is unstable (fixed-point periods diverge
after ~11 periods: the cylinder wake sheds), so shooting to 1e-8 from the free
stream takes far more sweeps than a bounded benchmark run; the full
time-to-gradient at 1e-8 is measured on the 8x24 p=1 workload (section
'ttg').

Extra sections (--sections, comma-separated, or 'all'): 'tiles' (forward
apply tile timings), 'mixed' (the step with FP32 and BF16 operator copies),
'batched' (instances on concurrent contexts), 'learned' (the learned warm
start and the combined learned + mixed-precision + block-Krylov form), 'ttg'
(the time to gradient on the 8x24 p=1 workload, compared with a
block-Krylov adjoint, one-workgroup stage solves and graph replay),
'ttg32' (the time to gradient on the 32x96 p=3 workload, shooting from
coarse orbits prolonged 8x24 p=1 -> 16x48 p=2 -> 32x96 p=3; several
minutes), 'batched' (32 instances on the 16x48 p=2 workload with five
right-hand sides each, by default), 'oracle-sweeps' (the oracle's sweeps on
the 8x24 workload on 1 and all host threads).  --solver-comparison runs only the shooting-solver comparison;
--spmv-only runs only the isolated applies used for hardware counters;
--ttg-only [--graph 1] only the plain 8x24 time to gradient (for profiling).

Prints progress on stderr and one JSON line on stdout.  --gpus N > 1 is
refused: the benchmark measures one GPU.
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("PA_VERBOSE", "1")   # progress lines from the library (stderr)

from paper_1512_00616_amd import inputs  # noqa: E402

HBM_PEAK_GBS = 8000.0
# hardware-counter traffic per launch of the FP64 stage-operator applies on
# the 32x96 p=3 workload (FETCH_SIZE and WRITE_SIZE calibrated against a
# plain copy; profiles/k_ahat_32x96_p3.md); valid for those kernels as
# measured, to be re-taken when they change
TRAFFIC_BYTES = {"pa::k_ahat_fwd<10, double, double, 0>": 243.4e6, "pa::k_ahat_tr_m<10>": 253.8e6}
# the forward apply as launched by the benchmark step: default tile shape
# (four 16-byte chunks per lane task); pa_config.autotune picks among 1, 2, 4
FWD_KERNEL = "pa::k_ahat_fwd<10, double, double, 0>"


def spmv_bytes(Nr, Nth, p, mat_bytes=8, vec_bytes=8, nrhs=1):
    """Algorithmic bytes of one apply of the preconditioned stage operator
    y = Ahat x = x + (A P^{-1} - I) x: every stored off-diagonal block once
    (two per interior face; the diagonal blocks are the identity), x and y
    once per right-hand side carried by the launch."""
    np_ = (p + 1) * (p + 2) // 2
    b = 4 * np_
    Ne = 2 * Nr * Nth
    n_int_faces = 3 * Ne // 2 - Nth          # wall and far-field edges are unpaired
    Nu = Ne * b
    return 2 * n_int_faces * b * b * mat_bytes + nrhs * 2 * Nu * vec_bytes


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(work, counts, mu):
    """The oracle timed on the host cores on a bounded sample of the same
    workload: at the three stages of the first step, one residual, one
    complex-step Jacobian and one block-Jacobi GMRES stage solve (seeded
    right-hand side) at the benchmark discretisation; the step time is
    composed from the mean unit times and the GPU step's own counts."""
    from oracle.oracle import Oracle
    ci = cpu_info()
    nthreads = min(ci["nproc"], 16)
    o = Oracle(lin_solver=1, lin_rtol=1e-10, nthreads=nthreads, **work)
    o.set_params(mu)
    u = o.freestream()
    t_res = t_jac = t_sol = 0.0
    its = 0
    rhs = inputs.random_vectors(o.Nu, 3, seed=7)
    a_ii = 0.4358665215084590          # the tableau's diagonal coefficient
    for i in (1, 2, 3):
        t0 = time.perf_counter()
        o.residual(1, i, u)
        t1 = time.perf_counter()
        J = o.jacobian(1, i, u)
        t2 = time.perf_counter()
        _, lin0 = o.counters()
        o.stage_solve(J, a_ii / work["Nt"], o.mass(rhs[i - 1]))
        t3 = time.perf_counter()
        _, lin1 = o.counters()
        t_res += t1 - t0
        t_jac += t2 - t1
        t_sol += t3 - t2
        its += lin1 - lin0
    o.close()
    t_res /= 3
    t_jac /= 3
    its = max(its, 1)
    t_it = t_sol / its
    est = counts["residuals"] * t_res + counts["jacobians"] * t_jac + counts["gmres_its"] * t_it
    dofs = counts["stage_solves"] * o.Nu / est
    return {
        "value": dofs, "unit": "DOF/s", "cores": nthreads, "kind": "oracle",
        "cpu_model": ci["model"], "nproc": ci["nproc"], "step_s": est, "composed": True,
        "sample_s": t_res * 3 + t_jac * 3 + t_sol,
        "sample": ("at the three stages of step 1 of the 32x96 p=3 workload: a residual (mean %.3f s) and a "
                   "complex-step Jacobian (mean %.2f s) on %d threads, and a block-Jacobi GMRES stage solve "
                   "(serial; %d iterations in all, %.4f s per iteration); step time composed with the GPU "
                   "step's counts (%d residuals, %d Jacobians, %d GMRES iterations, %d stage solves)"
                   % (t_res, t_jac, nthreads, its, t_it, counts["residuals"], counts["jacobians"],
                      counts["gmres_its"], counts["stage_solves"])),
    }


def time_to_gradient(pa, mu):
    """Full Alg. 4 on the 8x24 p=1, 20-step workload: shooting from the free
    stream (+ seeded N(0,1e-3) perturbation) to ||u^(Nt) - u0||_2 <= 1e-8, then
    the periodic adjoint gradient of both QoIs at relative 1e-8; then the
    same run with every stage solve in one workgroup (pa_config.wg_solve)
    and with the stage-GMRES iterations replayed from captured graphs
    (pa_config.graph) for comparison."""
    work = inputs.WORKLOADS["circle-8x24-p1-nt20"]
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, **work, **inputs.PHYSICS)
    s.set_params(mu)
    pert = inputs.perturbation(s.Nu, seed=1)
    s.set_freestream(pert)
    t0 = time.perf_counter()
    rep = s.shoot(tol=1e-8, eta=1e-3, maxit=30)
    t1 = time.perf_counter()
    q, dJ, arep = s.adjoint_gradient(rtol=1e-8)
    t = time.perf_counter() - t0
    # after the timed region: leading Floquet multipliers of the orbit
    # (Arnoldi with 40 tangent sweeps)
    ritz, _ = s.floquet(k=40, seed=13)
    u_per = s.get_state(0)
    s.close()
    # and the same periodic adjoint with one block Krylov space for both QoIs
    b = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, block_krylov=1,
                  **work, **inputs.PHYSICS)
    b.set_params(mu)
    b.set_state(u_per)
    b.primal_period()
    tb = time.perf_counter()
    _, dJb, brep = b.adjoint_gradient(rtol=1e-8)
    tb = time.perf_counter() - tb
    b.close()
    k = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, wg_solve=1, **work,
                  **inputs.PHYSICS)
    k.set_params(mu)
    k.set_freestream(inputs.perturbation(k.Nu, seed=1))
    tk = time.perf_counter()
    krep = k.shoot(tol=1e-8, eta=1e-3, maxit=30)
    _, dJk, _ = k.adjoint_gradient(rtol=1e-8)
    tk = time.perf_counter() - tk
    k.close()
    log("ttg: stage solves in one workgroup: %.1f s" % tk)
    # the same run with the stage-GMRES iterations replayed from captured
    # graphs (pa_config.graph): the same kernels, bitwise equal results
    h = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, graph=1, **work,
                  **inputs.PHYSICS)
    h.set_params(mu)
    h.set_freestream(inputs.perturbation(h.Nu, seed=1))
    th = time.perf_counter()
    hrep = h.shoot(tol=1e-8, eta=1e-3, maxit=30)
    _, dJh, _ = h.adjoint_gradient(rtol=1e-8)
    th = time.perf_counter() - th
    h.close()
    log("ttg: stage-GMRES iterations replayed from graphs: %.1f s" % th)
    return {"workload": "circle-8x24-p1-nt20", "seconds": t, "newton": rep.newton_its,
            "tangent_sweeps": rep.krylov_its, "periodicity": rep.res, "adjoint_krylov": list(arep.krylov_its),
            "counts": {"primal_sweeps": rep.primal_sweeps, "tangent_sweeps": rep.krylov_its,
                       "backward_rhs": arep.rhs_sweeps},
            "adjoint_seconds": t0 + t - t1, "qoi": list(q), "dJdmu": dJ.tolist(),
            "block_adjoint": {"krylov": list(brep.krylov_its), "sweeps": brep.sweeps, "seconds": tb,
                              "rel_res": list(brep.rel_res),
                              "dJdmu_rel_diff": float(np.abs(dJb - dJ).max() / np.abs(dJ).max())},
            "floquet_leading": [[float(z.real), float(z.imag)] for z in ritz[:4]],
            "workgroup_form": {"seconds": tk, "newton": krep.newton_its, "tangent_sweeps": krep.krylov_its,
                               "dJdmu_rel_diff": float(np.abs(dJk - dJ).max() / np.abs(dJ).max())},
            "graph_form": {"seconds": th, "newton": hrep.newton_its, "tangent_sweeps": hrep.krylov_its,
                           "dJdmu_bitwise_equal": bool(np.array_equal(dJh, dJ))}}


def ttg_only(pa, mu, graph):
    """The plain Alg. 4 run of time_to_gradient alone (8x24 p=1, 20 steps;
    graph = pa_config.graph), with its counts."""
    work = inputs.WORKLOADS["circle-8x24-p1-nt20"]
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, graph=graph, **work,
                  **inputs.PHYSICS)
    s.set_params(mu)
    s.set_freestream(inputs.perturbation(s.Nu, seed=1))
    t0 = time.perf_counter()
    rep = s.shoot(tol=1e-8, eta=1e-3, maxit=30)
    q, dJ, arep = s.adjoint_gradient(rtol=1e-8)
    t = time.perf_counter() - t0
    s.close()
    return {"workload": "circle-8x24-p1-nt20", "graph": graph, "seconds": t, "newton": rep.newton_its,
            "tangent_sweeps": rep.krylov_its, "shoot_stage_gmres": rep.stage_gmres_its,
            "adjoint_stage_gmres": arep.stage_gmres_its, "adjoint_krylov": list(arep.krylov_its),
            "dJdmu": dJ.tolist()}


def solver_comparison(pa, mu, descent_maxit=150):
    """Shooting solvers on the 8x24 p=1, 20-step workload (Sec. 2.2: Alg. 1,
    Newton-Krylov shooting, and minimisation of 1/2 ||R||^2 by L-BFGS or
    steepest descent), from the free stream with the seeded N(0, 1e-3)
    perturbation after m = 0, 1, 5 fixed-point periods used as nonlinear
    preconditioning.  Every method runs to ||u^(Nt) - u0||_2 <= 1e-8
    (Newton-Krylov with GMRES forcing 1e-2, 1e-3, 1e-4; L-BFGS with 10
    pairs and steepest descent capped at descent_maxit iterations); the plain
    fixed-point iteration runs 60 periods.  Sweep counts include the m
    preconditioning periods."""
    work = inputs.WORKLOADS["circle-8x24-p1-nt20"]
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, **work, **inputs.PHYSICS)
    s.set_params(mu)
    pert = inputs.perturbation(s.Nu, seed=1)
    tol = 1e-8
    methods = [("newton-gmres eta=1e-2", 1e-2, None), ("newton-gmres eta=1e-3", 1e-3, None),
               ("newton-gmres eta=1e-4", 1e-4, None), ("l-bfgs m=10", None, 10), ("steepest descent", None, 0)]
    runs = []
    for m in (0, 1, 5):
        for name, eta, mem in methods:
            s.set_freestream(pert)
            t0 = time.perf_counter()
            row = {"m": m, "method": name}
            try:
                r_pre = s.fixed_point(m) if m else None
                if eta is not None:
                    rep = s.shoot(tol=tol, eta=eta, maxit=30, allow_unconverged=True)
                else:
                    rep = s.shoot_descent(tol=tol, memory=mem, maxit=descent_maxit, allow_unconverged=True)
                row.update({"converged": bool(rep.res <= tol), "iterations": rep.newton_its,
                            "primal_sweeps": rep.primal_sweeps + m,
                            "tangent_sweeps": rep.krylov_its if eta is not None else 0,
                            "adjoint_sweeps": rep.krylov_its if eta is None else 0,
                            "res_start": rep.res0, "res": rep.res, "res_after_fixed_point": r_pre})
            except pa.PaError as e:
                row.update({"converged": False, "error": str(e)})
            row["seconds"] = time.perf_counter() - t0
            log("solvers: m=%d %-22s %s" % (m, name, {k: row[k] for k in row if k in ("iterations", "res",
                                                                                   "seconds", "error")}))
            runs.append(row)
    s.set_freestream(pert)
    fp = [s.fixed_point(1) for _ in range(60)]
    s.close()
    return {"workload": "circle-8x24-p1-nt20", "tol": tol, "runs": runs,
            "fixed_point_residuals": fp[:10] + fp[10::5]}


def apply_tiles(pa, work):
    """Autotuning of the forward apply's tile shape (chunks of 16 bytes per
    lane task) on the first stored operator of a short run on the benchmark
    mesh; the benchmark step itself uses the default shape (4)."""
    phys = dict(inputs.PHYSICS, T=0.03)
    s = pa.Solver(autotune=1, **dict(work, Nt=3), **phys)
    s.set_params(np.zeros(3))
    s.set_freestream()
    s.primal_period()
    q, us = s.tuning()
    s.close()
    return {"chosen_chunks_per_task": q, "us_per_launch": dict(zip(("1", "2", "4"), us)),
            "default_chunks_per_task": 4}


def learned(pa, args):
    """Learned warm start on the 8x24 p=1, 20-step workload: periodic orbits
    for seeded training parameters (seed 5) by concurrent contexts, POD + MLP
    trained on the device, then time to gradient (shooting to 1e-8 and both
    QoIs' periodic adjoint gradients at 1e-8) on held-out draws (seed 55)
    from the free stream and from the predicted state (with the free-stream
    fallback rule).  The combined form repeats the warm start in a context
    with FP32 mixed-precision stage solves and one block Krylov space for
    both QoIs' adjoints (several right-hand sides), at the same 1e-8
    tolerances; its speedup is taken against the plain FP64 run from the
    free stream."""
    name = "circle-8x24-p1-nt20"
    work = dict(inputs.WORKLOADS[name], **inputs.PHYSICS)
    mu_tr = inputs.warmstart_params(args.learned_train, seed=5)
    t0 = time.perf_counter()
    _, _, per, states = pa.batch_gradients(mu_tr, workers=8, shoot_maxit=30, shoot_tol=1e-8, shoot_eta=1e-3,
                                           return_states=True, keep_going=True, **work)
    t_gen = time.perf_counter() - t0
    ok = np.isfinite(per)
    s = pa.Solver(**work)
    t0 = time.perf_counter()
    modes = min(args.learned_modes, int(ok.sum()) - 1)
    loss = s.ws_train(mu_tr[ok], states[ok], modes=modes, width=256, epochs=3000, lr=1e-3, seed=5)
    t_train = time.perf_counter() - t0
    comb, comb_err = None, None
    try:
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "ws.bin")
            s.ws_save(path)
            comb = pa.Solver(precision=pa.PREC_FP32, block_krylov=1, **work)
            comb.ws_load(path)
    except pa.PaError as e:
        comb_err = str(e)
    tests = []
    for mu in inputs.warmstart_params(args.learned_test, seed=55):
        row = {"mu": [float(x) for x in mu]}
        for mode in ("free_stream", "warm"):
            s.set_params(mu)
            t0 = time.perf_counter()
            try:
                if mode == "warm":
                    rep, fb = s.ws_shoot(tol=1e-8, eta=1e-3, maxit=30)
                    row["fell_back"] = fb
                else:
                    s.set_freestream()
                    rep = s.shoot(tol=1e-8, eta=1e-3, maxit=30)
                _, dJ, _ = s.adjoint_gradient(rtol=1e-8)
                row[mode] = {"seconds": time.perf_counter() - t0, "newton": rep.newton_its,
                             "tangent_sweeps": rep.krylov_its, "periodicity": rep.res}
                row[mode + "_dJ"] = dJ
            except pa.PaError as e:
                row[mode] = {"failed": str(e), "seconds": time.perf_counter() - t0}
        if comb is not None:
            comb.set_params(mu)
            t0 = time.perf_counter()
            try:
                rep, fb = comb.ws_shoot(tol=1e-8, eta=1e-3, maxit=30)
                _, dJc, arc = comb.adjoint_gradient(rtol=1e-8)
                row["combined"] = {"seconds": time.perf_counter() - t0, "newton": rep.newton_its,
                                   "tangent_sweeps": rep.krylov_its, "periodicity": rep.res, "fell_back": fb,
                                   "adjoint_krylov": list(arc.krylov_its)}
                if "free_stream_dJ" in row:
                    b = row["free_stream_dJ"]
                    row["combined"]["dJdmu_rel_diff_vs_fp64"] = float(np.abs(dJc - b).max() / np.abs(b).max())
                    row["combined"]["speedup_vs_fp64_free_stream"] = (row["free_stream"]["seconds"]
                                                                      / row["combined"]["seconds"])
            except pa.PaError as e:
                row["combined"] = {"failed": str(e), "seconds": time.perf_counter() - t0}
        if "free_stream_dJ" in row and "warm_dJ" in row:
            a, b = row.pop("warm_dJ"), row.pop("free_stream_dJ")
            row["dJdmu_rel_diff"] = float(np.abs(a - b).max() / np.abs(b).max())
        row.pop("warm_dJ", None)
        row.pop("free_stream_dJ", None)
        tests.append(row)
    s.close()
    if comb is not None:
        comb.close()
    return {"workload": name, "training_orbits": int(ok.sum()), "training_draws": args.learned_train,
            "generation_s": t_gen, "train_s": t_train, "final_loss": loss,
            "model": "POD %d modes + MLP 4-256-256-256-%d (inputs h0, theta0, phi, Mach; tanh, FP32, MFMA "
                     "layer products, Adam 3000 full-batch steps)" % (modes, modes),
            "combined_form": "learned warm start + FP32 mixed-precision stage solves + block Krylov adjoint",
            "combined_setup_error": comb_err, "held_out": tests}


def time_to_gradient_fine(pa, mu, args):
    """Alg. 4 on the 32x96 p=3, 100-step workload from a coarse orbit: the
    8x24 p=1 and 16x48 p=2 discretisations (same physics, same 100 steps per
    period) are shot to periodicity in turn, each from the previous level's
    periodic state prolonged to its nodes (the first from the free stream),
    and the prolonged 16x48 orbit starts the 32x96 shooting to
    ||u^(Nt) - u0||_2 <= 1e-8; then both QoIs' periodic adjoint gradients at
    relative 1e-8.  Shooting eta 1e-3; stage solves block-Jacobi GMRES(30)
    at 1e-10.  Times per level; the fine-level time to gradient is the
    32x96 shooting plus its adjoint."""
    levels = [dict(Nr=8, Nth=24, p=1), dict(Nr=16, Nth=48, p=2), dict(Nr=32, Nth=96, p=3)]
    out = {"workload": "circle-32x96-p3-nt100", "levels": []}
    prev, u_prev = None, None
    t_all = time.perf_counter()
    for k, lev in enumerate(levels):
        cfgd = dict(lev, Nt=100, **inputs.PHYSICS)
        s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=120, **cfgd)
        s.set_params(mu)
        t0 = time.perf_counter()
        if prev is None:
            s.set_freestream()
        else:
            s.set_state(s.prolong_from(prev, u_prev))
        fine = k == len(levels) - 1
        try:
            rep = s.shoot(tol=1e-8, eta=1e-3, maxit=args.ttg32_maxit, allow_unconverged=True)
        except pa.PaError as e:   # e.g. the line search finds no decrease: report where it stopped
            out["levels"].append({"Nr": lev["Nr"], "Nth": lev["Nth"], "p": lev["p"], "Nu": s.Nu,
                                  "shoot_s": time.perf_counter() - t0, "error": str(e)})
            log("ttg32: level %dx%d p=%d: %s" % (lev["Nr"], lev["Nth"], lev["p"], e))
            s.close()
            break
        t_shoot = time.perf_counter() - t0
        res, kry, lam = rep.history()
        entry = {"Nr": lev["Nr"], "Nth": lev["Nth"], "p": lev["p"], "Nu": s.Nu, "shoot_s": t_shoot,
                 "newton": rep.newton_its, "tangent_sweeps": rep.krylov_its, "primal_sweeps": rep.primal_sweeps,
                 "res0": rep.res0, "res": rep.res, "res_hist": res.tolist(), "krylov_hist": kry.tolist(),
                 "step_hist": lam.tolist(), "stage_gmres": rep.stage_gmres_its}
        log("ttg32: level %dx%d p=%d shot in %.1f s: %d Newton, %d tangent sweeps, |R| %.3e -> %.3e" %
            (lev["Nr"], lev["Nth"], lev["p"], t_shoot, rep.newton_its, rep.krylov_its, rep.res0, rep.res))
        if not rep.res <= 1e-8:
            out["levels"].append(entry)
            s.close()
            break
        if fine:
            t1 = time.perf_counter()
            q, dJ, arep = s.adjoint_gradient(rtol=1e-8)
            t_adj = time.perf_counter() - t1
            entry.update({"adjoint_s": t_adj, "adjoint_krylov": list(arep.krylov_its),
                          "adjoint_rel_res": list(arep.rel_res), "qoi": q.tolist(), "dJdmu": dJ.tolist(),
                          "converged": bool(rep.res <= 1e-8)})
            out["fine_time_to_gradient_s"] = t_shoot + t_adj
            log("ttg32: adjoint gradient in %.1f s" % t_adj)
        else:
            prev, u_prev = cfgd, s.get_state(0)
        out["levels"].append(entry)
        s.close()
    out["total_s"] = time.perf_counter() - t_all
    return out


def batched(pa, args):
    """Many kinematic instances (seeded h0 ~ U[0.1,0.5], theta0 ~ U[0,30 deg],
    phi ~ U[0,pi]) on the 16x48 p=2, 60-step workload: the same bounded
    per-instance step as the main benchmark (one Newton-Krylov shooting step
    with a 6-vector basis), then five right-hand sides per instance: both
    QoIs' periodic adjoints (one backward sweep carries both) and the three
    parameter tangents of the direct gradient (one forward sweep carries all
    three), at relative 1e-8; run one after another on one context and by
    concurrent contexts inside the library (pa_batch_gradients); instances
    per second of each."""
    name = "circle-16x48-p2-nt60"
    work = dict(inputs.WORKLOADS[name], **inputs.PHYSICS)
    mu = inputs.batch_params(args.batch, seed=4)
    kw = dict(shoot_maxit=1, allow_unconverged=True, max_krylov=args.krylov, direct=True, **work)
    t0 = time.perf_counter()
    q1, g1, _, d1 = pa.batch_gradients(mu, workers=1, **kw)
    t_seq = time.perf_counter() - t0
    log("batched: %d instances one after another: %.1f s" % (args.batch, t_seq))
    t0 = time.perf_counter()
    qb, gb, _, db = pa.batch_gradients(mu, workers=args.batch_workers, **kw)
    t_bat = time.perf_counter() - t0
    log("batched: %d instances on %d concurrent contexts: %.1f s" % (args.batch, args.batch_workers, t_bat))
    return {"workload": name, "instances": args.batch, "workers": args.batch_workers,
            "step": "1 NK shooting step (basis %d) + periodic adjoint gradient of both QoIs + direct gradient "
                    "(3 parameter tangents): 5 right-hand sides per instance" % args.krylov,
            "sequential_s": t_seq, "batched_s": t_bat,
            "instances_per_s": args.batch / t_bat, "sequential_instances_per_s": args.batch / t_seq,
            "speedup": t_seq / t_bat,
            "bitwise_equal": bool(np.array_equal(g1, gb) and np.array_equal(q1, qb) and np.array_equal(d1, db))}


def cpu_info():
    """Host CPU model and the cores visible to this process."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"model": model, "nproc": avail}


def oracle_sweeps(mu, nthreads, counts=None):
    """The oracle's sweeps on the 8x24 p=1, 20-step workload on nthreads host
    threads: one primal period from the seeded perturbed free stream, one
    tangent sweep and one unforced backward sweep about it (block-Jacobi
    GMRES(30) stage solves at 1e-10).  With the GPU run's sweep counts of the
    whole method (shooting to 1e-8 and both QoIs' periodic adjoints), the
    oracle's time to gradient is composed from these unit times."""
    from oracle.oracle import Oracle
    work = inputs.WORKLOADS["circle-8x24-p1-nt20"]
    o = Oracle(lin_solver=1, lin_rtol=1e-10, newton_atol=1e-10, nthreads=nthreads, **work)
    o.set_params(mu)
    u0 = o.freestream(inputs.perturbation(o.Nu, seed=1))
    v = inputs.random_vectors(o.Nu, 1, seed=7)[0]
    t0 = time.perf_counter()
    o.primal_period(u0)
    t1 = time.perf_counter()
    o.tangent(v)
    t2 = time.perf_counter()
    o.adjoint(v)
    t3 = time.perf_counter()
    o.close()
    r = {"threads": nthreads, "primal_period_s": t1 - t0, "tangent_sweep_s": t2 - t1, "adjoint_sweep_s": t3 - t2}
    if counts:
        r["composed_time_to_gradient_s"] = (counts["primal_sweeps"] * r["primal_period_s"]
                                            + counts["tangent_sweeps"] * r["tangent_sweep_s"]
                                            + counts["backward_rhs"] * r["adjoint_sweep_s"])
        r["composed_from"] = counts
    return r


def roofline_entry(name, ms, launches, skipped, nbytes):
    """Achieved bandwidth of one kernel from the sampled HIP-event times over
    the timed steps: algorithmic bytes per working launch / (total time /
    working launches).  Launches that exited at once (their GMRES system had
    converged) move no bytes; their short time stays in the total."""
    work = launches - skipped
    if work <= 0 or ms <= 0:
        return None
    avg_s = ms / work / 1e3
    ach = nbytes / avg_s / 1e9
    return {"kernel": name, "total_ms": ms, "launches": launches, "launches_skipped": skipped,
            "bytes_per_launch": nbytes, "avg_launch_us": avg_s * 1e6, "achieved_gbs": ach,
            "frac": ach / HBM_PEAK_GBS, "avg_launch_us_all": ms / launches * 1e3}


SECTIONS = ("tiles", "mixed", "batched", "learned", "ttg", "ttg32", "oracle-sweeps")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steps (at most; see --budget-s)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up steps (at most; see --warmup-budget-s)")
    ap.add_argument("--budget-s", type=float, default=100.0,
                    help="wall-time budget of the timed steps: a further step starts only if the mean step time "
                         "says it ends inside the budget (at least one step is timed); the steps actually timed "
                         "are reported")
    ap.add_argument("--warmup-budget-s", type=float, default=45.0,
                    help="the same budget for the warm-up steps (at least one when --warmup > 0)")
    ap.add_argument("--krylov", type=int, default=6, help="outer Krylov basis cap of the step")
    ap.add_argument("--lin-guess", type=int, default=0, choices=(0, 1),
                    help="tangent and adjoint stage solves start from the neighbouring step's solution")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections", default="",
                    help="comma-separated extra sections after the headline step: " + ", ".join(SECTIONS)
                         + " (or 'all'); none by default")
    ap.add_argument("--batch", type=int, default=32,
                    help="instances of the 16x48 p=2 batched comparison (section 'batched')")
    ap.add_argument("--batch-workers", type=int, default=4)
    ap.add_argument("--ttg32-maxit", type=int, default=12,
                    help="Newton steps allowed per level of section 'ttg32'")
    ap.add_argument("--learned-train", type=int, default=16,
                    help="periodic orbits that train the warm start on the 8x24 p=1 workload (section 'learned')")
    ap.add_argument("--learned-test", type=int, default=2, help="held-out parameter draws of the warm-start test")
    ap.add_argument("--learned-modes", type=int, default=16, help="POD modes of the warm-start model")
    ap.add_argument("--ttg-only", action="store_true",
                    help="only the plain Alg. 4 on the 8x24 p=1 workload (for profiling), then exit")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="with --ttg-only: replay the stage-GMRES iterations from captured graphs")
    ap.add_argument("--spmv-only", action="store_true",
                    help="short run for hardware counters: a 3-stage period on the 32x96 p=3 mesh, then timed "
                         "launches of the preconditioned stage operator and of a plain copy")
    ap.add_argument("--solver-comparison", action="store_true",
                    help="only the shooting-solver comparison on the 8x24 p=1 workload (about 15 minutes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the sweeps are sequential in time and the library runs on a single "
              "MI355X; --gpus above 1 is not supported", file=sys.stderr)
        return 2
    sections = set(SECTIONS) if args.sections.strip() == "all" else \
        {x.strip() for x in args.sections.split(",") if x.strip()}
    bad = sections - set(SECTIONS)
    if bad:
        print("unknown sections: %s (known: %s)" % (sorted(bad), ", ".join(SECTIONS)), file=sys.stderr)
        return 2

    from paper_1512_00616_amd import pa

    name = "circle-32x96-p3-nt100"
    work = inputs.WORKLOADS[name]
    mu = np.array(inputs.MU_NOMINAL)
    if args.solver_comparison:
        print(json.dumps({"solver_comparison": solver_comparison(pa, mu)}), flush=True)
        return 0
    if args.spmv_only:
        print(json.dumps(spmv_only(pa, work)), flush=True)
        return 0
    if args.ttg_only:
        print(json.dumps(ttg_only(pa, mu, args.graph)), flush=True)
        return 0

    out, dJ64 = run_step(pa, name, work, mu, args, pa.PREC_FP64)
    if not args.no_cpu_baseline:
        log("oracle sample on the host")
        c = out.pop("_cpu_counts")
        try:
            out["cpu_baseline"] = cpu_baseline(work, c, mu)
        except Exception as e:  # report, do not fail the benchmark
            out["cpu_baseline"] = {"value": None, "error": str(e)}
    out.pop("_cpu_counts", None)
    if "tiles" in sections:
        out["apply_tiles"] = apply_tiles(pa, work)
    if "mixed" in sections:
        # the same step with the mixed-precision stage solves (FP64 refinement
        # to the same tolerances): wall time and gradient against the FP64 run
        out["mixed_precision"] = {}
        for prec, tag in ((pa.PREC_FP32, "fp32"), (pa.PREC_BF16, "bf16")):
            log("mixed precision (%s operator copy, FP32 inner GMRES)" % tag)
            m, dJm = run_step(pa, name, work, mu, args, prec)
            out["mixed_precision"][tag] = {
                "ms_per_step": m["ms_per_step"], "value": m["value"], "unit": "DOF/s", "steps": m["steps"],
                "speedup_vs_fp64": out["ms_per_step"] / m["ms_per_step"],
                "dJdmu_rel_diff_vs_fp64": float(np.abs(dJm - dJ64).max() / np.abs(dJ64).max()),
                "counts": m["counts"], "kernels_ms": m["kernels_ms"],
                "spmv_lo": m["spmv_lo"],
            }
    if "batched" in sections:
        log("batched instances on the 16x48 p=2 workload")
        out["batched"] = batched(pa, args)
    if "learned" in sections:
        log("learned warm start on the 8x24 p=1 workload")
        out["learned_warm_start"] = learned(pa, args)
    if "ttg" in sections:
        log("time to gradient on the 8x24 p=1 workload")
        out["time_to_gradient"] = time_to_gradient(pa, mu)
    if "ttg32" in sections:
        log("time to gradient on the 32x96 p=3 workload from prolonged coarse orbits")
        out["time_to_gradient_32x96"] = time_to_gradient_fine(pa, mu, args)
    if "oracle-sweeps" in sections:
        log("oracle sweeps on the 8x24 p=1 workload (1 thread, all threads)")
        ci = cpu_info()
        cnt = out.get("time_to_gradient", {}).get("counts")
        out["oracle_sweeps"] = {"cpu": ci, "runs": [oracle_sweeps(mu, 1, cnt),
                                                    oracle_sweeps(mu, min(ci["nproc"], 16), cnt)]}
    print(json.dumps(out), flush=True)
    return 0


def spmv_only(pa, work):
    """Isolated applies for hardware counters: the same mesh, degree and time
    step (dt = 0.01) as the workload, three steps of a motionless cylinder
    (stores the operators of 9 stages), then timed launches of the stored
    first-stage operator (forward, transposed, two right-hand sides) in FP64,
    of its FP32 and BF16 copies, and of a plain device copy."""
    phys = dict(inputs.PHYSICS, T=0.03)
    outj = {}
    for prec, tag in ((pa.PREC_FP32, "fp32"), (pa.PREC_BF16, "bf16")):
        s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, precision=prec,
                      **dict(work, Nt=3), **phys)
        s.set_params(np.zeros(3))
        s.set_freestream()
        s.primal_period()
        if prec == pa.PREC_FP32:
            fwd = s.bench_spmv(20)
            trn = s.bench_spmv(20, transpose=True)
            trm = s.bench_spmv(20, transpose=True, nrhs=2)
            fwm = s.bench_spmv(20, transpose=False, nrhs=3)
            nbytes = spmv_bytes(work["Nr"], work["Nth"], work["p"])
            outj.update({"spmv_us": fwd * 1e3, "spmv_t_us": trn * 1e3, "spmv_bytes": nbytes,
                         "spmv_gbs": nbytes / (fwd * 1e-3) / 1e9, "spmv_t_gbs": nbytes / (trn * 1e-3) / 1e9,
                         "spmv_tm2_us": trm * 1e3,
                         "spmv_tm2_gbs": spmv_bytes(work["Nr"], work["Nth"], work["p"], nrhs=2) / (trm * 1e-3) / 1e9,
                         "spmv_fm3_us": fwm * 1e3,
                         "spmv_fm3_gbs": spmv_bytes(work["Nr"], work["Nth"], work["p"], nrhs=3) / (fwm * 1e-3) / 1e9})
        lo = s.bench_spmv_lo(20)
        lot = s.bench_spmv_lo(20, transpose=True)
        lb = spmv_bytes(work["Nr"], work["Nth"], work["p"], 4 if tag == "fp32" else 2, 4)
        outj.update({"spmv_%s_us" % tag: lo * 1e3, "spmv_%s_t_us" % tag: lot * 1e3, "spmv_%s_bytes" % tag: lb,
                     "spmv_%s_gbs" % tag: lb / (lo * 1e-3) / 1e9})
        if prec == pa.PREC_BF16:
            cp_ms, cp_bytes = s.bench_copy(20)
            outj.update({"copy_us": cp_ms * 1e3, "copy_bytes": cp_bytes,
                         "copy_gbs": 2 * cp_bytes / (cp_ms * 1e-3) / 1e9})
        s.close()
    return outj


def run_step(pa, name, work, mu, args, precision):
    """Warm-up, then the timed steps, on a fresh context of the given
    stage-solve precision, both within their wall-time budgets; returns the
    report and dJ/dmu of the last step."""
    t_setup = time.perf_counter()
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=args.krylov,
                  precision=precision, lin_guess=args.lin_guess, **work, **inputs.PHYSICS)
    s.set_params(mu)
    setup_s = time.perf_counter() - t_setup
    log("setup %.1f s, %.1f GB on the device" % (setup_s, s.device_bytes / 1e9))

    def step():
        s.set_freestream()
        rep = s.shoot(tol=1e-8, eta=1e-3, maxit=1, allow_unconverged=True)
        q, dJ, arep = s.adjoint_gradient(rtol=1e-8)
        return rep, q, dJ, arep

    def budgeted(k_max, budget, tag):
        res, t0 = [], time.perf_counter()
        while len(res) < k_max:
            el = time.perf_counter() - t0
            if res and el + el / len(res) > budget:
                break
            res.append(step())
            log("%s step %d: %.1f s" % (tag, len(res), time.perf_counter() - t0))
        return res, time.perf_counter() - t0

    warm, _ = budgeted(args.warmup, args.warmup_budget_s, "warm-up")
    s.set_timing(True)
    results, t_run = budgeted(max(args.steps, 1), args.budget_s, "timed")
    ids = ("spmv", "spmv_t", "spmv_m", "spmv_tm", "spmv_lo", "mdot", "gmupd", "precond", "jacobian", "residual",
           "blockinv")
    kt = {k: s.kernel_time(getattr(pa, "PA_K_" + k.upper())) for k in ids}
    ksk = {k: s.kernel_skipped(getattr(pa, "PA_K_" + k.upper())) for k in ids}
    kvec = {k: s.kernel_vectors(getattr(pa, "PA_K_" + k.upper())) for k in ("mdot", "gmupd")}
    s.set_timing(False)
    nsteps = len(results)
    step_s = t_run / nsteps
    rep, q, dJ, arep = results[-1]
    nst = 3 * work["Nt"]
    gmres_its = rep.stage_gmres_its + arep.stage_gmres_its
    # stage solves of the step: primal Newton corrections, 3 Nt per tangent
    # sweep, 3 Nt per right-hand side of each backward sweep (the two QoIs'
    # adjoints ride in the same sweeps)
    stage_solves = rep.stage_newton_its + nst * (rep.krylov_its + arep.rhs_sweeps)
    Nu = s.Nu
    Nr, Nth, p = work["Nr"], work["Nth"], work["p"]
    fwd_name = FWD_KERNEL if Nr * Nth > 0 else None
    cand = [roofline_entry(fwd_name, kt["spmv"][0], kt["spmv"][1], ksk["spmv"], spmv_bytes(Nr, Nth, p)),
            roofline_entry("pa::k_ahat_tr<%d, double, double>" % ((p + 1) * (p + 2) // 2), kt["spmv_t"][0],
                           kt["spmv_t"][1], ksk["spmv_t"], spmv_bytes(Nr, Nth, p)),
            # the two QoIs' adjoints in one transposed launch
            roofline_entry("pa::k_ahat_tr_m<%d>" % ((p + 1) * (p + 2) // 2), kt["spmv_tm"][0], kt["spmv_tm"][1],
                           ksk["spmv_tm"], spmv_bytes(Nr, Nth, p, nrhs=2)),
            roofline_entry("pa::k_ahat_fwd_m<%d>" % ((p + 1) * (p + 2) // 2), kt["spmv_m"][0], kt["spmv_m"][1],
                           ksk["spmv_m"], spmv_bytes(Nr, Nth, p, nrhs=3))]
    cand = [c for c in cand if c]
    dom = max(cand, key=lambda c: c["total_ms"])
    full = (Nr, Nth, p) == (32, 96, 3)
    traffic = TRAFFIC_BYTES.get(dom["kernel"]) if full else None
    # the Krylov vector kernels: one pass over the basis columns each; their
    # bytes depend on the column index: the library counts the length-Nu
    # vectors their working launches read or wrote, so the mean algorithmic
    # bytes per working launch and the achieved bandwidth follow
    vec = {}
    for k in ("mdot", "gmupd"):
        work_k = max(kt[k][1] - ksk[k], 1)
        nbytes = kvec[k] * Nu * 8 / work_k
        avg_us = kt[k][0] / work_k * 1e3
        vec[k] = {"total_ms": kt[k][0], "launches": kt[k][1], "launches_skipped": ksk[k], "avg_launch_us": avg_us,
                  "vectors": kvec[k], "bytes_per_launch": nbytes,
                  "achieved_gbs": nbytes / (avg_us * 1e-6) / 1e9 if avg_us > 0 else None,
                  "frac": nbytes / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS if avg_us > 0 else None}
    lo_bytes = spmv_bytes(Nr, Nth, p, 4 if precision == pa.PREC_FP32 else 2, 4)
    ms_lo, n_lo = kt["spmv_lo"]
    work_lo = n_lo - ksk["spmv_lo"]
    out = {
        "metric": "stage-solve DOF/s (periodic adjoint hot path, 32x96 p=3)",
        "value": stage_solves * Nu / step_s,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": len(warm),
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "budget_s": args.budget_s,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == pa.PREC_FP64 else ("f32+f64" if precision == pa.PREC_FP32 else "bf16+f32+f64"),
        "data": "synthetic",
        "config": {"workload": name, **work, "mu": list(mu), "stage_gmres": "block-Jacobi GMRES(30) rtol 1e-10",
                   "newton_atol": 1e-10, "outer_krylov_cap": args.krylov, "shoot_eta": 1e-3, "adj_rtol": 1e-8,
                   "lin_guess": args.lin_guess},
        "roofline": {"bound": "hbm", "achieved": dom["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["frac"], "traffic": traffic, **dom},
        "applies": cand,
        "gmres_vector_kernels": vec,
        "spmv_lo": ({"avg_launch_us": ms_lo / work_lo * 1e3, "launches": n_lo, "launches_skipped": ksk["spmv_lo"],
                     "bytes_per_launch": lo_bytes, "achieved_gbs": lo_bytes / (ms_lo / work_lo * 1e-3) / 1e9}
                    if work_lo > 0 else None),
        "kernels_ms": {k: v[0] for k, v in kt.items()},
        "counts": {"stage_solves": stage_solves, "stage_newton": rep.stage_newton_its, "stage_gmres": gmres_its,
                   "primal_sweeps": rep.primal_sweeps, "tangent_sweeps": rep.krylov_its,
                   "backward_sweeps": arep.sweeps, "backward_rhs": arep.rhs_sweeps,
                   "adjoint_krylov": list(arep.krylov_its)},
        "periodicity": {"res0": rep.res0, "res_after_step": rep.res},
        "qoi": list(q), "dJdmu": dJ.tolist(),
        "setup_s": setup_s,
        "device_gb": s.device_bytes / 1e9,
        "_cpu_counts": {"residuals": kt["residual"][1] // nsteps,
                        "jacobians": kt["jacobian"][1] // nsteps,
                        "gmres_its": gmres_its, "stage_solves": stage_solves},
    }
    if precision == pa.PREC_FP64:
        out.pop("spmv_lo")
    s.close()
    return out, dJ


if __name__ == "__main__":
    sys.exit(main())
