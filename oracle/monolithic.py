"""Dense monolithic solve of the fully discrete periodic problem's
linearisation and of its adjoint, for tiny meshes.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the tests to
check the sweep-based periodic adjoint (Alg. 3, Alg. 4) and the direct
gradient against one dense linear solve over every unknown of a period.

Sec. 3 writes the time-periodic fully discrete problem as one system
(eq. abs-govern-disc) in the unknowns w = (u^(0), ..., u^(Nt), k_i^(n)):

    rt^(0) = u^(0) - u^(Nt)                                  = 0
    rt^(n) = u^(n) - u^(n-1) - sum_i b_i k_i^(n)             = 0,  n = 1..Nt
    R_i^(n) = M k_i^(n) - dt r(u_i^(n), mu, t_{n-1} + c_i dt) = 0,
              u_i^(n) = u^(n-1) + sum_{j<=i} a_ij k_j^(n).

Its Jacobian dRt/dw is assembled here as a dense matrix from the oracle's
stage Jacobians dr/du(u_i^(n)) (complex step), the mass matrix and the DIRK
tableau, with no sweep, no Krylov method and no reuse of the oracle's
adjoint recurrences.  Sec. 3.1 then gives

    adjoint (eq. uns-disc-adj):     (dRt/dw)^T psi = (dF/dw)^T,
    gradient (eq. funcl-grad-nosens): dF/dmu = dF/dmu|explicit - psi^T dRt/dmu,

and the direct method solves (dRt/dw) dw = -dRt/dmu, dF/dmu = dF/dmu|explicit
+ dF/dw dw.  F is the time-averaged QoI of the solver-consistent reading
(1/T) sum_n sum_i dt b_i f(u_i^(n), mu, t), so it depends on w through the
stage states only.  dRt/dmu is nonzero only in the stage rows:
-dt dr/dmu(u_i^(n)).

The trajectory (u^(n), k_i^(n), u_i^(n)) is the oracle's stored periodic
primal period; the linear algebra is numpy (dense LU via numpy.linalg.solve).
"""
import numpy as np

from . import oracle as O


def _layout(o):
    Nt, Nu = o.Nt, o.Nu
    n_u = (Nt + 1) * Nu

    def iu(n):           # block of u^(n), n = 0..Nt
        return slice(n * Nu, (n + 1) * Nu)

    def ik(n, i):        # block of k_i^(n), n = 1..Nt, i = 1..3
        s = n_u + ((n - 1) * 3 + (i - 1)) * Nu
        return slice(s, s + Nu)

    return n_u + 3 * Nt * Nu, iu, ik


def _mass_matrix(o):
    return np.stack([o.mass(e) for e in np.eye(o.Nu)], axis=1)


def _bsr_dense(o, blk):
    """dr/du as a dense Nu x Nu matrix from the BSR blocks (column by column
    through the oracle's block product)."""
    return np.stack([o.bsr_apply(blk, e) for e in np.eye(o.Nu)], axis=1)


def assemble(o, T=1.0):
    """Dense dRt/dw, dRt/dmu [.., 3], dF/dw [2, ..] and the explicit dF/dmu
    [2, 3] about the oracle's stored trajectory (call primal_period first)."""
    A, b, c = O.dirk_tableau()
    Nt, Nu = o.Nt, o.Nu
    dt = T / Nt
    n, iu, ik = _layout(o)
    Jw = np.zeros((n, n))
    Jmu = np.zeros((n, 3))
    Fw = np.zeros((2, n))
    Fmu = np.zeros((2, 3))
    I = np.eye(Nu)
    M = _mass_matrix(o)
    # periodicity rows (first block row): u^(0) - u^(Nt)
    Jw[iu(0), iu(0)] += I
    Jw[iu(0), iu(Nt)] -= I
    for m in range(1, Nt + 1):
        # state update rows: u^(n) - u^(n-1) - sum_i b_i k_i^(n)
        Jw[iu(m), iu(m)] += I
        Jw[iu(m), iu(m - 1)] -= I
        for i in range(1, 4):
            Jw[iu(m), ik(m, i)] -= b[i - 1] * I
        for i in range(1, 4):
            ui = o.traj(0, m, i)
            dr = _bsr_dense(o, o.traj_jacobian(m, i))
            # stage rows: M k_i - dt r(u_i), u_i = u^(n-1) + sum_{j<=i} a_ij k_j
            row = ik(m, i)
            Jw[row, ik(m, i)] += M
            Jw[row, iu(m - 1)] -= dt * dr
            for j in range(1, i + 1):
                Jw[row, ik(m, j)] -= dt * A[i - 1, j - 1] * dr
            Jmu[row, :] = -dt * o.dr_dmu(m, i, ui).T
            # F = (1/T) sum dt b_i f(u_i): derivatives through u_i
            _, dfdu, dfdmu = o.qoi(m, i, ui, derivs=True)
            wgt = dt * b[i - 1] / T
            Fw[:, iu(m - 1)] += wgt * dfdu
            for j in range(1, i + 1):
                Fw[:, ik(m, j)] += wgt * A[i - 1, j - 1] * dfdu
            Fmu += wgt * dfdmu
    return Jw, Jmu, Fw, Fmu


def residual(o, T=1.0):
    """The rows of eq. abs-govern-disc evaluated on the stored trajectory (all
    zero up to the Newton and shooting tolerances on a periodic orbit)."""
    A, b, c = O.dirk_tableau()
    Nt = o.Nt
    dt = T / Nt
    out = [o.traj(2, 0) - o.traj(2, Nt)]
    for m in range(1, Nt + 1):
        k = [o.traj(1, m, i) for i in range(1, 4)]
        out.append(o.traj(2, m) - o.traj(2, m - 1) - sum(b[i] * k[i] for i in range(3)))
        for i in range(1, 4):
            ui = o.traj(0, m, i)
            out.append(o.mass(k[i - 1]) - dt * o.residual(m, i, ui))
    return np.concatenate(out)


def gradients(o, T=1.0):
    """(adjoint gradient, direct gradient, multipliers psi [2, n]) of both
    QoIs from one dense assembly: eq. uns-disc-adj solved with the transposed
    matrix, eq. funcl-grad-nosens for dF/dmu; the direct method with the
    matrix itself."""
    Jw, Jmu, Fw, Fmu = assemble(o, T)
    psi = np.linalg.solve(Jw.T, Fw.T).T
    g_adj = Fmu - psi @ Jmu
    dw = np.linalg.solve(Jw, -Jmu)
    g_dir = Fmu + Fw @ dw
    return g_adj, g_dir, psi
