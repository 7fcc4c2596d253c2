"""Pins of the FP64 POD reference (oracle/pod.py, method of snapshots) by
construction: snapshots built from a known mean, known orthonormal modes and
snapshot coefficients with zero mean over the snapshots and mutually
orthogonal rows of known norms.  Then the centred snapshot matrix is
D = C^T Psi with C C^T = diag(s_j^2), so the Gram matrix D D^T has the
eigenvalues s_j^2, the POD modes are the psi_j (up to sign), and the
coefficients are C -- a mistake in the centring, the Gram product's
orientation, the eigen-ordering or the mode normalisation fails one of
these."""
import numpy as np

from oracle import pod


def _construct(S=12, N=300, k=4, seed=3):
    g = np.random.default_rng(seed)
    Psi = np.linalg.qr(g.standard_normal((N, k)))[0].T            # k orthonormal modes (rows)
    # coefficients: rows orthogonal to each other and to the all-ones vector
    B = np.linalg.qr(np.column_stack([np.ones(S), g.standard_normal((S, k))]))[0][:, 1:].T
    s = np.array([5.0, 3.0, 1.5, 0.5])[:k]
    C = s[:, None] * B                                          # C C^T = diag(s^2), C 1 = 0
    mean = g.standard_normal(N)
    X = mean[None, :] + C.T @ Psi
    return X, mean, Psi, s, C


def test_pod_recovers_constructed_modes():
    X, mean, Psi, s, C = _construct()
    m, modes, eig, coef = pod.pod(X, 4)
    assert np.allclose(m, mean, atol=1e-13)
    assert np.allclose(eig, s ** 2, rtol=1e-12)
    aligned = pod.align_signs(modes, Psi)
    assert np.allclose(aligned, Psi, atol=1e-12)
    sg = np.sign(np.sum(modes * Psi, axis=1))
    assert np.allclose(coef * sg[:, None], C, atol=1e-12)


def test_modes_orthonormal_and_snapshots_reconstructed():
    X, mean, Psi, s, C = _construct(S=9, N=200, k=3, seed=8)
    m, modes, eig, coef = pod.pod(X, 3)
    assert np.allclose(modes @ modes.T, np.eye(3), atol=1e-12)
    assert np.allclose(m[None, :] + coef.T @ modes, X, atol=1e-12)
    assert np.all(np.diff(eig) <= 0)


def test_mode_count_is_capped_by_the_snapshots():
    g = np.random.default_rng(1)
    X = g.standard_normal((5, 40))
    m, modes, eig, coef = pod.pod(X, 10)
    assert modes.shape == (4, 40) and eig.shape == (4,) and coef.shape == (4, 5)
    # the centred snapshots of 5 states span 4 dimensions: all of them are reproduced
    assert np.allclose(m[None, :] + coef.T @ modes, X, atol=1e-12)
