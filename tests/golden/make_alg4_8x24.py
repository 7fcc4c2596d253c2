"""Writes alg4_8x24_p1_nt20.npz: the oracle's whole method (Alg. 4) on the
8x24 O-grid, p = 1, 20 DIRK3 steps per period, nominal kinematics, from the
free stream plus the seeded N(0, 1e-3) perturbation (seed 1):

  * Newton-Krylov shooting (Alg. 2, Sec. 2.2) to ||u^(Nt) - u0||_2 <= 1e-11
    with GMRES forcing 1e-10;
  * both QoIs' periodic adjoints (Alg. 3, Sec. 3.2) at relative 1e-13 and the
    gradient of eq. funcl-grad-nosens-dirk;
  * the direct (periodic tangent) gradient at relative 1e-13.

Stage solves: block-Jacobi GMRES(30) at relative 1e-13, Newton to 1e-12.
Calls only the oracle; run from the repository root:
    python tests/golden/make_alg4_8x24.py
(about 15-30 minutes on 8 host threads).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import build  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from paper_1512_00616_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "alg4_8x24_p1_nt20.npz")


def main():
    build.build()
    work = inputs.WORKLOADS["circle-8x24-p1-nt20"]
    mu = np.array(inputs.MU_NOMINAL)
    o = Oracle(lin_solver=1, lin_rtol=1e-13, newton_atol=1e-12, **work, **inputs.PHYSICS)
    o.set_params(mu)
    u0 = o.freestream(inputs.perturbation(o.Nu, seed=1))
    t0 = time.time()
    us, rep = o.shoot(u0, tol=1e-11, eta=1e-10, maxit=30, max_krylov=300)
    print("shoot: %d Newton, %d Krylov, |R| = %.3e, %.0f s" % (rep.outer_its, rep.krylov_its, rep.final_res,
                                                              time.time() - t0), flush=True)
    _, q, res = o.primal_period(us)
    G = np.stack([o.periodic_adjoint(k, rtol=1e-13, max_krylov=400)[0] for k in (0, 1)])
    print("adjoint gradient", G.tolist(), "%.0f s" % (time.time() - t0), flush=True)
    T = o.tangent_gradient(rtol=1e-13, max_krylov=400)
    print("direct gradient", T.tolist(), "%.0f s" % (time.time() - t0), flush=True)
    np.savez_compressed(OUT, mu=mu, u_periodic=us, qoi=q, periodicity=res, dJdmu_adjoint=G, dJdmu_direct=T,
                        newton=rep.outer_its)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
