"""Stage-GMRES iterations replayed from captured HIP graphs
(pa_config.graph) against the same context type launching every kernel
from the host: the replays run the same kernels with the same arguments in
the same order, so every result is bitwise equal.  Each run replays its
graphs hundreds of times with the library's own eager launches, copies and
synchronisations in between, and every stage solve's output feeds the
next, so a replay that went wrong once would show in the compared results.
The parity tests against the oracle run the graph form too
(`tests/test_gpu_parity.py`, `tests/test_gpu_parity_p3.py`)."""
import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

MU = np.array(inputs.MU_NOMINAL)


def run_alg4(graph, work, maxit):
    from paper_1512_00616_amd import pa
    s = pa.Solver(gmres_restart=30, lin_rtol=1e-10, newton_atol=1e-10, max_krylov=100, graph=graph, **work,
                  **inputs.PHYSICS)
    s.set_params(MU)
    s.set_freestream(inputs.perturbation(s.Nu, seed=1))
    rep = s.shoot(tol=1e-8, eta=1e-3, maxit=maxit, allow_unconverged=True)
    u0 = s.get_state(0)
    q, dJ, arep = s.adjoint_gradient(rtol=1e-6)
    tg, its = s.tangent_gradient(rtol=1e-6)
    out = dict(u0=u0, q=q, dJ=dJ, tg=tg, res=rep.res, gmres=rep.stage_gmres_its, krylov=rep.krylov_its,
               adj=list(arep.krylov_its), tits=list(its))
    s.close()
    return out


@pytest.mark.parametrize("name,maxit", [("circle-8x24-p1-nt20", 2), ("circle-2x6-p3-nt16", 1)])
def test_graph_replay_bitwise_equal_to_host_launches(name, maxit):
    work = inputs.WORKLOADS[name] if name in inputs.WORKLOADS else dict(Nr=2, Nth=6, p=3, Nt=16)
    print("graph replay case", name, flush=True)
    a = run_alg4(0, work, maxit)
    b = run_alg4(1, work, maxit)
    assert a["gmres"] == b["gmres"] and a["krylov"] == b["krylov"]
    assert a["adj"] == b["adj"] and a["tits"] == b["tits"]
    assert a["res"] == b["res"]
    for k in ("u0", "q", "dJ", "tg"):
        assert np.array_equal(a[k], b[k]), k


def test_graph_stage_solves_all_restart_chunks():
    # single stage solves, forward and transposed (graphs of either kind
    # replayed in turn), against host launches
    from paper_1512_00616_amd import pa
    from oracle import oracle as O
    o = O.Oracle(Nr=3, Nth=8, p=2, Nt=2, lin_solver=0)
    o.set_params(MU)
    u = o.freestream(inputs.perturbation(o.Nu, seed=18, sigma=1e-2))
    J = o.jacobian(1, 2, u)
    rhs = inputs.random_vectors(o.Nu, 1, seed=19)[0]
    c = 0.5 * 0.4358665215084590
    res = {}
    for graph in (0, 1):
        g = pa.Solver(Nr=3, Nth=8, p=2, Nt=2, lin_rtol=1e-13, gmres_restart=30, graph=graph)
        g.set_params(MU)
        res[graph] = [g.stage_solve(J, c, rhs, transpose=tr) for tr in (False, True, False)]
        g.close()
    for (xa, ia), (xb, ib) in zip(res[0], res[1]):
        assert ia == ib and ia > 5
        assert np.array_equal(xa, xb)
