"""Block GMRES for the outer solves with several right-hand sides (the two
QoIs' periodic adjoints of Alg. 3, the three parameter tangents of the
direct gradient): one Krylov space shared by all systems (pa_config
block_krylov = 1) against one space per system in lockstep, on the same
periodic orbit.  The block space after k sweeps contains every single
system's k-dimensional space and block GMRES minimises each system's
residual over it, so it needs no more sweeps."""
import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

TINY = dict(Nr=2, Nth=6, p=1, Nt=8, lin_rtol=1e-13, newton_atol=1e-12)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


@pytest.fixture(scope="module")
def pair():
    from paper_1512_00616_amd import pa
    a = pa.Solver(**TINY)
    b = pa.Solver(block_krylov=1, **TINY)
    for s in (a, b):
        s.set_params(np.array(inputs.MU_NOMINAL))
    a.set_freestream(inputs.perturbation(a.Nu, seed=1))
    a.shoot(tol=1e-12, eta=1e-8, maxit=30)
    b.set_state(a.get_state(0))
    b.primal_period()
    yield a, b
    a.close()
    b.close()


def test_block_adjoint_gradient_matches_lockstep_and_oracle(pair):
    from oracle.oracle import Oracle
    a, b = pair
    qa, ga, ra = a.adjoint_gradient(rtol=1e-13)
    qb, gb, rb = b.adjoint_gradient(rtol=1e-13)
    assert np.array_equal(qa, qb)                      # the same stored trajectory
    assert rel(gb, ga) <= 1e-10
    # Alg. 3 of the oracle (one Krylov space per QoI, exact stage solves)
    # about the same orbit
    o = Oracle(lin_solver=0, newton_atol=1e-12, **{k: TINY[k] for k in ("Nr", "Nth", "p", "Nt")})
    o.set_params(np.array(inputs.MU_NOMINAL))
    o.primal_period(a.get_state(0))
    go = np.stack([o.periodic_adjoint(q, rtol=1e-13)[0] for q in (0, 1)])
    assert rel(gb, go) <= 1e-10
    to = o.tangent_gradient(rtol=1e-13)
    gt, _ = b.tangent_gradient(rtol=1e-13)
    assert rel(gt, to) <= 1e-10
    o.close()
    ka, kb = list(ra.krylov_its), list(rb.krylov_its)
    assert kb[0] == kb[1] >= 1                         # one block iteration = one sweep for both QoIs
    # no more sweeps than the slower lockstep system (one more at most where
    # rounding moves the residual estimate across the threshold)
    assert kb[0] <= max(ka) + 1
    assert max(rb.rel_res) <= 1e-13
    assert rb.sweeps == 2 + kb[0]                      # g_F sweep, Krylov sweeps, final sweep


def test_block_tangent_gradient_matches_lockstep(pair):
    a, b = pair
    ga, ia = a.tangent_gradient(rtol=1e-13)
    gb, ib = b.tangent_gradient(rtol=1e-13)
    assert rel(gb, ga) <= 1e-10
    assert ib[0] == ib[1] == ib[2] >= 1
    assert ib[0] <= max(ia) + 1
