"""Learned warm start: the device perceptron kernels against the FP64
reference, and shooting from the predicted state against shooting from the
free stream on held-out parameters (same periodic orbit, no more Newton
steps, a closer start; free-stream fallback when the first step fails)."""
import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

TINY = dict(Nr=2, Nth=6, p=1, Nt=8)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


@pytest.mark.parametrize("width,batch", [(256, 24), (32, 1), (48, 37)])
def test_mlp_kernels_match_fp64_reference(width, batch):
    from paper_1512_00616_amd import pa
    from oracle import mlp
    g = np.random.default_rng(11 + width)
    dims = [3, width, width, width, 16]
    parts = []
    for l in range(4):
        a = np.sqrt(6.0 / (dims[l] + dims[l + 1]))
        parts += [g.uniform(-a, a, dims[l + 1] * dims[l]), 0.1 * g.standard_normal(dims[l + 1])]
    p = np.concatenate(parts).astype(np.float32)
    X = g.standard_normal((3, batch)).astype(np.float32)
    T = g.standard_normal((16, batch)).astype(np.float32)
    lg, gg = pa.dbg_mlp(p, X, T, width)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), dims, X.astype(np.float64), T.astype(np.float64))
    # FP32 kernels against FP64: sums of at most 256 products per entry
    assert abs(lg - lo) <= 1e-5 * lo
    assert np.abs(gg - go).max() <= 1e-5 * np.abs(go).max()


@pytest.fixture(scope="module")
def trained(tmp_path_factory):
    from paper_1512_00616_amd import pa
    mu_tr = inputs.warmstart_params(24, seed=5)
    _, _, per, states = pa.batch_gradients(mu_tr, workers=8, shoot_maxit=30, shoot_tol=1e-10, shoot_eta=1e-6,
                                           return_states=True, keep_going=True, lin_rtol=1e-12,
                                           newton_atol=1e-11, **TINY)
    ok = np.isfinite(per)
    assert ok.sum() >= 16
    s = pa.Solver(lin_rtol=1e-12, newton_atol=1e-11, **TINY)
    loss = s.ws_train(mu_tr[ok], states[ok], modes=16, width=256, epochs=3000, lr=1e-3, seed=5)
    assert loss < 1e-3   # normalised targets start near 1
    path = tmp_path_factory.mktemp("ws") / "model.bin"
    s.ws_save(path)
    yield s, path
    s.close()


def test_warm_start_reaches_the_same_orbit_in_fewer_steps(trained):
    s, _ = trained
    mu_te = inputs.warmstart_params(4, seed=55)
    saved = 0
    for i in range(len(mu_te)):
        s.set_params(mu_te[i])
        s.set_freestream()
        u_fs = s.get_state(0)
        r0 = s.shoot(tol=1e-10, eta=1e-6, maxit=30)
        u_per = s.get_state(0)
        s.ws_predict(mu_te[i])
        u_pr = s.get_state(0)
        r1, fell_back = s.ws_shoot(tol=1e-10, eta=1e-6, maxit=30)
        assert r1.res <= 1e-10
        assert rel(s.get_state(0), u_per) <= 1e-8
        if fell_back:
            assert r1.newton_its >= r0.newton_its   # the failed first step plus the free-stream run
        else:
            assert np.linalg.norm(u_pr - u_per) < np.linalg.norm(u_fs - u_per)
            assert r1.newton_its <= r0.newton_its
            saved += r0.newton_its - r1.newton_its
    assert saved >= 2


def test_saved_model_predicts_the_same_bits(trained):
    from paper_1512_00616_amd import pa
    s, path = trained
    mu = inputs.warmstart_params(1, seed=55)[0]
    s.set_params(mu)
    s.ws_predict(mu)
    a = s.get_state(0)
    s2 = pa.Solver(**TINY)
    s2.set_params(mu)
    with pytest.raises(pa.PaError):
        s2.ws_predict(mu)                      # no model yet
    s2.ws_load(path)
    s2.ws_predict(mu)
    assert np.array_equal(s2.get_state(0), a)
    s2.close()
