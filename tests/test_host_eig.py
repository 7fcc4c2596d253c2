"""The library's host-side dense eigen-solvers, called through the C ABI
without a GPU: the complex shifted QR behind the Floquet multipliers
(pa_floquet) and the cyclic Jacobi behind the warm start's POD basis."""
import numpy as np
import pytest

from paper_1512_00616_amd import pa


def match(a, b):
    """max distance between two multisets of complex numbers (greedy)"""
    b = list(b)
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - y) for y in b]))
        worst = max(worst, abs(z - b.pop(k)))
    return worst


def test_hessenberg_eigenvalues_of_a_companion_matrix():
    # the companion matrix of prod (x - r_k) is upper Hessenberg and has the
    # roots r_k as eigenvalues (closed form)
    roots = np.array([1.22 + 0.53j, 1.22 - 0.53j, 0.9, -0.5 + 0.2j, -0.5 - 0.2j, 0.3, 0.05])
    c = np.real(np.poly(roots))
    n = len(roots)
    H = np.zeros((n, n))
    H[0, :] = -c[1:]
    H[np.arange(1, n), np.arange(n - 1)] = 1.0
    ev = pa.dbg_hess_eig(H)
    assert match(ev, roots) <= 1e-10
    assert np.all(np.diff(np.abs(ev)) <= 1e-12)       # by decreasing modulus


@pytest.mark.parametrize("n,seed", [(40, 1), (7, 2), (1, 3), (200, 5)])   # 200: the Floquet count
def test_hessenberg_eigenvalues_match_numpy(n, seed):
    g = np.random.default_rng(seed)
    H = np.triu(g.standard_normal((n, n)), -1)
    ev = pa.dbg_hess_eig(H)
    ref = np.linalg.eigvals(H)
    assert match(ev, ref) <= 1e-10 * max(1.0, np.abs(ref).max())
    # entries below the subdiagonal are ignored
    H2 = H + np.tril(g.standard_normal((n, n)), -2)
    assert np.array_equal(pa.dbg_hess_eig(H2), ev)


def test_symmetric_eigenpairs():
    g = np.random.default_rng(4)
    B = g.standard_normal((30, 30))
    A = B @ B.T                                       # a Gram matrix, as in the POD
    w, V = pa.dbg_sym_eig(A)
    assert np.all(np.diff(w) <= 0)
    assert np.allclose(w, np.sort(np.linalg.eigvalsh(A))[::-1], rtol=0, atol=1e-11 * w[0])
    assert np.abs(V.T @ V - np.eye(30)).max() <= 1e-12
    assert np.abs(A @ V - V * w).max() <= 1e-11 * w[0]


def test_symmetric_eigenpairs_of_a_graded_gram_matrix():
    """The POD's Gram matrix at scale: 256 snapshots whose eigenvalues fall
    geometrically over 12 decades, as a snapshot set's do.  The leading 64
    eigenpairs (the warm start's largest basis) come out to 1e-10 relative
    each, with their modes."""
    g = np.random.default_rng(5)
    n, k = 256, 64
    Q = np.linalg.qr(g.standard_normal((n, n)))[0]
    lam = 1e4 * 10.0 ** (-np.linspace(0, 12, n))
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    w, V = pa.dbg_sym_eig(A)
    assert np.all(np.diff(w) <= 0)
    assert (np.abs(w[:k] - lam[:k]) / lam[:k]).max() <= 1e-10
    assert np.abs(np.sum(V[:, :k] * Q[:, :k], axis=0)).min() >= 1 - 1e-10
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12
    assert np.abs(A @ V - V * w).max() <= 1e-12 * lam[0]


def test_bad_arguments_raise():
    with pytest.raises(pa.PaError):
        pa.dbg_hess_eig(np.zeros((0, 0)))
    with pytest.raises(pa.PaError):
        pa.dbg_sym_eig(np.zeros((0, 0)))
