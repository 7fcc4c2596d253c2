"""Many kinematic instances through pa_batch_gradients: contexts running side
by side give the same bits as the same instances run one after another, and
the gradients -- by the periodic adjoint (two right-hand sides) and by the
direct method (three parameter tangents) -- agree with the CPU oracle."""
import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(Nr=2, Nth=6, p=1, Nt=8, lin_rtol=1e-13, newton_atol=1e-12)


def test_batch_equals_sequential_and_oracle():
    from paper_1512_00616_amd import pa
    from oracle.oracle import Oracle
    mu = inputs.batch_params(5, seed=4)
    opts = dict(shoot_maxit=20, shoot_tol=1e-12, shoot_eta=1e-12, adj_rtol=1e-13)
    qb, gb, pb, gdb = pa.batch_gradients(mu, workers=3, direct=True, **opts, **KW)
    assert np.all(pb <= 1e-12)
    # one context, instances one after another
    s = pa.Solver(**KW)
    for i in range(len(mu)):
        s.set_params(mu[i])
        s.set_freestream()
        rep = s.shoot(tol=opts["shoot_tol"], eta=opts["shoot_eta"], maxit=opts["shoot_maxit"])
        q, g, _ = s.adjoint_gradient(rtol=opts["adj_rtol"])
        gd, _ = s.tangent_gradient(rtol=opts["adj_rtol"])
        assert np.array_equal(q, qb[i]) and np.array_equal(g, gb[i]) and rep.res == pb[i]
        assert np.array_equal(gd, gdb[i])
    s.close()
    # instance 3 against the oracle
    o = Oracle(lin_solver=0, newton_atol=1e-12, **{k: KW[k] for k in ("Nr", "Nth", "p", "Nt")})
    o.set_params(mu[3])
    us, _ = o.shoot(o.freestream(), tol=1e-12, eta=1e-12, maxit=20, max_krylov=300)
    o.primal_period(us)
    go = np.stack([o.periodic_adjoint(q, rtol=1e-13)[0] for q in (0, 1)])
    assert np.abs(gb[3] - go).max() <= 1e-10 * np.abs(go).max()
    assert np.abs(gdb[3] - go).max() <= 1e-10 * np.abs(go).max()


def test_batch_rejects_bad_arguments():
    from paper_1512_00616_amd import pa
    with pytest.raises(pa.PaError):
        pa.batch_gradients(np.zeros((2, 3)), workers=0, **KW)
