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


# ---------------------------------------------------------------- POD, Mach input, prolongation
def _smooth_snapshots(s, mus, machs, seed):
    """snapshots = the free stream of each (mu, Mach) plus deviations from a
    few fixed directions with well separated amplitudes (so that the POD
    modes are well conditioned)"""
    from oracle.oracle import Oracle
    g = np.random.default_rng(seed)
    dirs = g.standard_normal((5, s.Nu))
    amp = 0.5 ** np.arange(5)
    out = []
    for mu, m in zip(mus, machs):
        o = Oracle(mach=m, **TINY)
        o.set_params(mu)
        fs = o.freestream()
        o.close()
        c = g.standard_normal(5) * amp
        out.append(fs + 1e-1 * (c @ dirs))
    return np.array(out), dirs


def test_pod_matches_fp64_reference():
    """Device POD (Gram matrix of the centred deviations, Jacobi eigenpairs,
    modes) against the oracle's FP64 method of snapshots on the same data,
    each snapshot's own free stream (its kinematics and Mach number)
    removed by each side independently."""
    from paper_1512_00616_amd import pa
    from oracle import pod
    from oracle.oracle import Oracle
    mus = inputs.warmstart_params(10, seed=5)
    machs = np.linspace(0.15, 0.25, 10)
    s = pa.Solver(**TINY)
    X, _ = _smooth_snapshots(s, mus, machs, seed=21)
    params = np.concatenate([mus, machs[:, None]], axis=1)
    s.ws_train(params, X, modes=4, width=16, epochs=10, lr=1e-3, seed=5)
    mean_g, modes_g, eig_g = s.ws_pod()
    dev = []
    for x, mu, m in zip(X, mus, machs):
        o = Oracle(mach=m, **TINY)
        o.set_params(mu)
        dev.append(x - o.freestream())
        o.close()
    mean_o, modes_o, eig_o, _ = pod.pod(np.array(dev), 4)
    assert len(eig_g) == 4
    # the deviations are differences of O(|X|) = 45 states and free streams,
    # so they carry an absolute rounding of about 1e-14 |X| on both sides
    scale = np.abs(X).max()
    assert np.abs(mean_g - mean_o).max() <= 1e-13 * scale
    assert rel(eig_g, eig_o) <= 1e-9
    assert rel(pod.align_signs(modes_g, modes_o), modes_o) <= 1e-8
    s.close()


def test_mach_input_reproduces_training_states(tmp_path):
    """Inputs (h0, theta0, phi, Mach): a model trained on snapshots of two Mach
    numbers, loaded into a context of either Mach number, predicts for a
    training input the training state (that Mach's free stream plus the POD
    expansion) up to the fitting error, far below the difference between
    the Mach numbers' states."""
    from paper_1512_00616_amd import pa
    mus = inputs.warmstart_params(8, seed=5)
    machs = np.array([0.2, 0.25] * 4)
    s = pa.Solver(**TINY)
    X, _ = _smooth_snapshots(s, mus, machs, seed=22)
    params = np.concatenate([mus, machs[:, None]], axis=1)
    loss = s.ws_train(params, X, modes=7, width=64, epochs=3000, lr=1e-3, seed=5)
    assert loss < 1e-2   # normalised coefficients start near 1
    path = tmp_path / "m.bin"
    s.ws_save(path)
    s.close()
    for i in (2, 3):
        c = pa.Solver(mach=float(machs[i]), **TINY)
        c.ws_load(path)
        c.set_params(mus[i])
        c.ws_predict(mus[i])
        err = np.abs(c.get_state(0) - X[i]).max()
        gap = np.abs(X[i] - X[i - 1]).max()
        assert err <= 2e-2 * gap, (i, err, gap)
        c.close()


# coefficients of 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3
POLY = np.array([1.0, 0.3, -0.2, 0.05, 0.02, -0.03, 0.004, -0.002, 0.001, 0.003])


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 3), (3, 3)])
def test_prolongation_is_exact_for_polynomials(pc, pf):
    """pa_prolong from a coarse O-grid (4x12) to the nested refined one (8x24):
    a field that is one polynomial of degree <= pc in X on every coarse
    element is reproduced at every fine node (each fine node lies in a
    coarse triangle, or between a coarse chord and the circle, where the
    same polynomial is extrapolated)."""
    from paper_1512_00616_amd import pa
    from oracle.oracle import Oracle
    coarse = dict(Nr=4, Nth=12, p=pc, Nt=2)
    oc = Oracle(**coarse)
    Xc, _ = oc.nodes()
    of = Oracle(Nr=8, Nth=24, p=pf, Nt=2)
    Xf, _ = of.nodes()
    k = (pc + 1) * (pc + 2) // 2

    def field(X):
        x, y = X[..., 0], X[..., 1]
        base = [np.ones_like(x), x, y, x * x, x * y, y * y, x ** 3, x * x * y, x * y * y, y ** 3][:k]
        out = np.zeros(X.shape[:-1] + (4,))
        for m in range(4):
            for j in range(k):
                out[..., m] += (m + 1) * POLY[j] * base[j]
        return out

    fine = pa.Solver(Nr=8, Nth=24, p=pf, Nt=2)
    uf = fine.prolong_from(coarse, field(Xc).ravel())
    assert rel(uf, field(Xf).ravel()) <= 1e-12
    fine.close()
    oc.close()
    of.close()
