"""The SQP subproblem behind pa_optimize (pa_dbg_qp3, host code):
minimise g.d + d^T B d / 2 subject to a.d = -c and lo <= d <= hi, with B
symmetric positive definite.  The problem is strictly convex, so the KKT
conditions characterise its unique minimiser: each returned point is
checked against them (feasibility; g + B d - lam a has a zero component on
every free variable, a non-negative one at a lower bound and a non-positive
one at an upper bound), and against scipy's SLSQP on the objective value.
An equality that no point of the box meets takes the nearest attainable
target."""
import numpy as np
import pytest
from scipy.optimize import minimize

from paper_1512_00616_amd import pa


def _spd(g, scale=1.0):
    Q = np.linalg.qr(g.standard_normal((3, 3)))[0]
    return scale * Q @ np.diag(g.uniform(0.1, 10.0, 3)) @ Q.T


def _check_kkt(B, g, a, t, lo, hi, d, lam, tol=1e-9):
    assert np.all(d >= lo - 1e-12) and np.all(d <= hi + 1e-12)
    if np.any(a):
        assert abs(a @ d - t) <= tol * (1 + np.abs(a).sum())
    r = g + B @ d - lam * a
    scale = 1 + np.abs(g).max() + np.abs(B).max()
    for i in range(3):
        at_lo = abs(d[i] - lo[i]) <= 1e-10
        at_hi = abs(d[i] - hi[i]) <= 1e-10
        if not at_lo and not at_hi:
            assert abs(r[i]) <= tol * scale, (i, r)
        elif at_lo and not at_hi:
            assert r[i] >= -tol * scale, (i, r)
        elif at_hi and not at_lo:
            assert r[i] <= tol * scale, (i, r)


def _slsqp(B, g, a, t, lo, hi):
    cons = [{"type": "eq", "fun": lambda d: a @ d - t, "jac": lambda d: a}] if np.any(a) else []
    best = None
    for x0 in (np.clip(np.zeros(3), lo, hi), (lo + hi) / 2, lo, hi):
        r = minimize(lambda d: g @ d + 0.5 * d @ B @ d, x0, jac=lambda d: g + B @ d, bounds=list(zip(lo, hi)),
                     constraints=cons, method="SLSQP", options=dict(ftol=1e-14, maxiter=500))
        if r.success and (best is None or r.fun < best.fun):
            best = r
    return best


@pytest.mark.parametrize("seed", range(40))
def test_random_subproblems_meet_kkt_and_match_slsqp(seed):
    g0 = np.random.default_rng(seed)
    B = _spd(g0, scale=10.0 ** g0.uniform(-2, 2))
    g = g0.standard_normal(3) * 10.0 ** g0.uniform(-1, 1)
    a = g0.standard_normal(3)
    if seed % 5 == 0:
        a[g0.integers(3)] = 0.0              # a variable outside the equality
    lo = -g0.uniform(0.05, 1.0, 3)
    hi = g0.uniform(0.05, 1.0, 3)
    c = g0.standard_normal() * 0.5
    d, lam = pa.dbg_qp3(B, g, a, c, lo, hi)
    amin = np.sum(np.where(a > 0, a * lo, a * hi))
    amax = np.sum(np.where(a > 0, a * hi, a * lo))
    t = min(max(-c, amin), amax)
    _check_kkt(B, g, a, t, lo, hi, d, lam)
    ref = _slsqp(B, g, a, t, lo, hi)
    assert ref is not None
    f = g @ d + 0.5 * d @ B @ d
    assert f <= ref.fun + 1e-9 * (1 + abs(ref.fun))


def test_interior_solution_is_the_equality_constrained_newton_step():
    B = np.diag([2.0, 4.0, 8.0])
    g = np.array([1.0, -1.0, 0.5])
    a = np.array([1.0, 1.0, 1.0])
    c = -0.1                                   # a.d = 0.1
    d, lam = pa.dbg_qp3(B, g, a, c, -np.ones(3), np.ones(3))
    K = np.block([[B, -a[:, None]], [a[None, :], np.zeros((1, 1))]])
    sol = np.linalg.solve(K, np.concatenate([-g, [0.1]]))
    assert np.allclose(d, sol[:3], atol=1e-14) and abs(lam - sol[3]) < 1e-13


def test_no_equality_is_a_box_constrained_minimum():
    B = np.eye(3)
    g = np.array([3.0, -0.2, -5.0])
    d, lam = pa.dbg_qp3(B, g, np.zeros(3), 0.0, -np.ones(3), np.ones(3))
    assert np.allclose(d, np.clip(-g, -1, 1), atol=1e-14) and lam == 0.0


def test_unreachable_equality_takes_the_nearest_target():
    B = np.eye(3)
    g = np.zeros(3)
    a = np.array([1.0, 2.0, -1.0])
    lo, hi = -0.1 * np.ones(3), 0.1 * np.ones(3)
    d, lam = pa.dbg_qp3(B, g, a, -10.0, lo, hi)      # a.d = 10 is out of reach: a.d = 0.4 at most
    assert np.allclose(d, [0.1, 0.1, -0.1], atol=1e-14)
    d, lam = pa.dbg_qp3(B, g, a, 10.0, lo, hi)
    assert np.allclose(d, [-0.1, -0.1, 0.1], atol=1e-14)
