"""Parity at p = 3 (40 x 40 blocks, the benchmark's block size) on a small
mesh: one primal period, the tangent and backward sweeps, and the periodic
adjoint (Alg. 3, both QoIs in the same backward sweeps: the two-system
transposed apply) and direct gradients (three parameter tangents in the
same forward sweeps: the three-system forward apply) about the same stored
trajectory, against the oracle.  The trajectory is one period from the
perturbed free stream, not a periodic orbit: the two-point boundary-value
problem of Sec. 3.1 is well posed about any trajectory (the machinery
reading of the one-period configuration), so both sides solve the same
linear problem."""
import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

MU = np.array(inputs.MU_NOMINAL)
KW = dict(Nr=2, Nth=6, p=3, Nt=16)   # 8 steps give the oracle a singular diagonal block at p = 3


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


TRAJ = [(1, 1), (7, 2), (16, 3)]


@pytest.fixture(scope="module")
def oracle_p3():
    """The oracle's side of every comparison below, computed once: it does
    not depend on the GPU's execution form, which is what the four GPU
    fixtures vary.  Same order of calls as on the GPU: one period, the
    sweeps, the periodic adjoints of both QoIs, the direct gradient."""
    from oracle.oracle import Oracle
    o = Oracle(lin_solver=1, lin_rtol=1e-13, newton_atol=1e-12, **KW)
    o.set_params(MU)
    u0 = o.freestream(inputs.perturbation(o.Nu, seed=1))
    uNt, qo, ro = o.primal_period(u0)
    v, w = inputs.random_vectors(o.Nu, 2, seed=7)
    ref = dict(uNt=uNt, qo=qo, ro=ro,
               traj={(n, i): o.traj(0, n, i) for n, i in TRAJ},
               tangent=o.tangent(v), adjoint=o.adjoint(w),
               forced=[o.adjoint(w, forced_qoi=q) for q in (0, 1)],
               periodic=np.stack([o.periodic_adjoint(q, rtol=1e-13)[0] for q in (0, 1)]),
               direct=o.tangent_gradient(rtol=1e-13))
    o.close()
    return ref


@pytest.fixture(scope="module", params=[(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
                ids=["kernels", "workgroup", "guess", "graph"])
def pair(request, oracle_p3):
    """wg_solve 0: the several-system applies k_ahat_tr_m / k_ahat_fwd_m
    and the GMRES vector kernels; 1: one workgroup per system and solve;
    guess: the linear sweeps start each stage solve from the neighbouring
    step's solution; graph: the GMRES iterations replayed from captured
    graphs"""
    from paper_1512_00616_amd import pa
    wg, guess, graph = request.param
    g = pa.Solver(lin_rtol=1e-13, newton_atol=1e-12, wg_solve=wg, lin_guess=guess, graph=graph, **KW)
    g.set_params(MU)
    g.set_freestream(inputs.perturbation(g.Nu, seed=1))
    qg, rg = g.primal_period()
    yield g, oracle_p3, (qg, rg)
    g.close()


def test_primal_period_p3(pair):
    g, ref, (qg, rg) = pair
    assert rel(g.get_state(1), ref["uNt"]) <= 1e-10
    assert rel(qg, ref["qo"]) <= 1e-10
    for n, i in TRAJ:
        assert rel(g.traj(0, n, i), ref["traj"][(n, i)]) <= 1e-10


def test_sweeps_p3(pair):
    g, ref, _ = pair
    v, w = inputs.random_vectors(g.Nu, 2, seed=7)
    assert rel(g.tangent_sweep(v), ref["tangent"]) <= 1e-10
    assert rel(g.adjoint_sweep(w), ref["adjoint"]) <= 1e-10
    for q in (0, 1):
        lg, gg = g.adjoint_sweep(w, forced_qoi=q)
        lo, go = ref["forced"][q]
        assert rel(lg, lo) <= 1e-10
        assert rel(gg, go) <= 1e-10


def test_two_system_adjoint_and_three_system_direct_gradient_p3(pair):
    g, ref, _ = pair
    _, dJ, rep = g.adjoint_gradient(rtol=1e-13)
    assert rep.rhs_sweeps > rep.sweeps                    # the QoIs share backward sweeps
    go = ref["periodic"]
    assert rel(dJ, go) <= 1e-10
    tg, its = g.tangent_gradient(rtol=1e-13)
    assert all(its > 0)
    to = ref["direct"]
    assert rel(tg, to) <= 1e-10
    assert rel(go, to) <= 1e-10
