"""FP64 reference of the proper orthogonal decomposition behind the learned
warm start (method of snapshots).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

Given S snapshot states x_1..x_S (columns of X, length N):
  1. the mean xbar = (1/S) sum_i x_i and the centred snapshots D = X - xbar;
  2. the S x S Gram matrix G = D^T D;
  3. its eigenpairs G v_j = lam_j v_j, lam_1 >= lam_2 >= ... (numpy.linalg.eigh);
  4. the modes psi_j = D v_j / sqrt(lam_j) (orthonormal in the Euclidean inner
     product) and the snapshot coefficients c_ji = psi_j^T d_i = sqrt(lam_j) v_ij.
The warm start predicts u0 = free stream + xbar + sum_j c_j psi_j for new
parameters, with the free stream of each snapshot's own parameters removed
before step 1 (so the centred data holds only the flow's deviation from the
uniform state).

Modes are determined up to sign; ``align_signs`` fixes a sign convention for
comparisons.
"""
import numpy as np


def pod(states, k):
    """states [S][N] (rows are snapshots); returns (mean [N], modes [k][N],
    eigenvalues [k], coefficients [k][S])."""
    X = np.asarray(states, dtype=np.float64)
    S = X.shape[0]
    mean = X.mean(axis=0)
    D = X - mean
    G = D @ D.T
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    k = min(k, S - 1)
    modes = (V[:, :k].T @ D) / np.sqrt(lam[:k])[:, None]
    coef = np.sqrt(lam[:k])[:, None] * V[:, :k].T
    return mean, modes, lam[:k], coef


def align_signs(modes, ref):
    """flip each mode so that its inner product with the matching reference
    mode is non-negative"""
    s = np.sign(np.sum(modes * ref, axis=1))
    s[s == 0] = 1.0
    return modes * s[:, None]
