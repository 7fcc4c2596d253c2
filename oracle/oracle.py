"""ctypes binding of the CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  Argument marshalling only; all arithmetic is in ``oracle.c``.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


class pao_config(C.Structure):
    _fields_ = [
        ("Nr", C.c_int32), ("Nth", C.c_int32), ("p", C.c_int32), ("Nt", C.c_int32),
        ("r_far", C.c_double), ("stretch", C.c_double),
        ("mach", C.c_double), ("re", C.c_double), ("gamma", C.c_double), ("pr", C.c_double),
        ("T", C.c_double), ("r_blend0", C.c_double), ("r_blend1", C.c_double),
        ("wall_is_farfield", C.c_int32), ("lin_solver", C.c_int32), ("gmres_restart", C.c_int32),
        ("lin_rtol", C.c_double), ("newton_atol", C.c_double), ("newton_maxit", C.c_int32),
        ("nthreads", C.c_int32),
    ]


class pao_krylov_report(C.Structure):
    _fields_ = [("outer_its", C.c_int32), ("krylov_its", C.c_int32), ("sweeps", C.c_int32),
                ("final_res", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle library not built: %s (run __graft_entry__.build())" % _LIB_PATH)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.pao_create.restype = P
        L.pao_create.argtypes = [C.POINTER(pao_config)]
        L.pao_destroy.argtypes = [P]
        L.pao_last_error.restype = C.c_char_p
        L.pao_last_error.argtypes = [P]
        L.pao_default_config.argtypes = [C.POINTER(pao_config)]
        L.pao_num_dofs.restype = C.c_int64
        L.pao_num_dofs.argtypes = [P]
        for fn in ("pao_num_elems", "pao_block_size", "pao_num_vol_points"):
            getattr(L, fn).restype = C.c_int32
            getattr(L, fn).argtypes = [P]
        L.pao_get_mesh.argtypes = [P, P, P, P, P]
        L.pao_get_nodes.argtypes = [P, P, P]
        L.pao_ref_tables.argtypes = [P, P, P, P, P]
        L.pao_dirk_tableau.argtypes = [P, P, P]
        L.pao_set_params.argtypes = [P, P]
        L.pao_gbar.argtypes = [P, C.c_int32, C.c_int32, P]
        L.pao_gcl_rhs.argtypes = [P, C.c_int32, C.c_int32, P]
        L.pao_freestream.argtypes = [P, P, P]
        L.pao_mass_apply.argtypes = [P, P, P]
        L.pao_residual.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.pao_jacobian.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.pao_dr_dmu.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.pao_qoi.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P]
        L.pao_bsr_apply.argtypes = [P, P, C.c_int32, P, P]
        L.pao_stage_solve.argtypes = [P, P, C.c_double, C.c_int32, P, P]
        L.pao_primal_period.argtypes = [P, P, P, P, P]
        L.pao_tangent_sweep.argtypes = [P, P, C.c_int32, P, P]
        L.pao_adjoint_sweep.argtypes = [P, P, C.c_int32, P, P]
        L.pao_shoot.argtypes = [P, P, C.c_double, C.c_double, C.c_int32, C.c_int32, P]
        L.pao_periodic_adjoint.argtypes = [P, C.c_int32, C.c_double, C.c_int32, P, P, P]
        L.pao_tangent_gradient.argtypes = [P, C.c_double, C.c_int32, P]
        L.pao_traj.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
        L.pao_traj_jacobian.argtypes = [P, C.c_int32, C.c_int32, P]
        L.pao_counters.argtypes = [P, P, P]
        L.pao_flux_vis.argtypes = [P, P, P, C.c_int32, P]
        L.pao_flux_h.argtypes = [P, P, P, C.c_double, P]
        L.pao_flux_lf.argtypes = [P, P, P, P, C.c_double, P]
        L.pao_face_lift.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int32, C.c_int32, P]
        L.pao_face_lift.restype = C.c_int
        for fn in ("pao_set_params", "pao_gbar", "pao_gcl_rhs", "pao_residual", "pao_jacobian",
                   "pao_dr_dmu", "pao_qoi", "pao_stage_solve", "pao_primal_period",
                   "pao_tangent_sweep", "pao_adjoint_sweep", "pao_shoot", "pao_periodic_adjoint",
                   "pao_tangent_gradient", "pao_traj", "pao_traj_jacobian"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def dirk_tableau():
    A = np.zeros(9)
    b = np.zeros(3)
    c = np.zeros(3)
    lib().pao_dirk_tableau(_ptr(A), _ptr(b), _ptr(c))
    return A.reshape(3, 3), b, c


class OracleError(RuntimeError):
    pass


class Oracle:
    """One discretised problem (mesh, physics, time grid) on the CPU."""

    def __init__(self, Nr=8, Nth=24, p=1, Nt=20, mach=0.2, re=1000.0, gamma=1.4, pr=0.72, T=1.0,
                 r_far=10.0, stretch=1.3, r_blend0=2.0, r_blend1=8.0, wall_is_farfield=False,
                 lin_solver=1, gmres_restart=30, lin_rtol=1e-12, newton_atol=1e-11,
                 newton_maxit=20, nthreads=0):
        cfg = pao_config()
        lib().pao_default_config(C.byref(cfg))
        for k, v in dict(Nr=Nr, Nth=Nth, p=p, Nt=Nt, mach=mach, re=re, gamma=gamma, pr=pr, T=T,
                         r_far=r_far, stretch=stretch, r_blend0=r_blend0, r_blend1=r_blend1,
                         wall_is_farfield=int(wall_is_farfield), lin_solver=lin_solver,
                         gmres_restart=gmres_restart, lin_rtol=lin_rtol,
                         newton_atol=newton_atol, newton_maxit=newton_maxit,
                         nthreads=nthreads).items():
            setattr(cfg, k, v)
        self.cfg = cfg
        self._c = lib().pao_create(C.byref(cfg))
        if not self._c:
            raise OracleError("pao_create failed (bad configuration)")
        self.Nu = lib().pao_num_dofs(self._c)
        self.Ne = lib().pao_num_elems(self._c)
        self.b = lib().pao_block_size(self._c)
        self.np = self.b // 4
        self.nq = lib().pao_num_vol_points(self._c)
        self.Nt = Nt
        self.Nr, self.Nth, self.p = Nr, Nth, p

    def close(self):
        if self._c:
            lib().pao_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc < 0:
            raise OracleError("oracle error %d: %s" % (rc, lib().pao_last_error(self._c).decode()))
        return rc

    def _vec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.Nu, (x.size, self.Nu)
        return x

    # mesh and tables
    def mesh(self):
        ev = np.zeros(self.Ne * 3, np.int32)
        en = np.zeros(self.Ne * 3, np.int32)
        tw = np.zeros(self.Ne * 3, np.int8)
        vxy = np.zeros((self.Nr + 1) * self.Nth * 2)
        lib().pao_get_mesh(self._c, _ptr(ev), _ptr(en), _ptr(tw), _ptr(vxy))
        return ev.reshape(-1, 3), en.reshape(-1, 3), tw.reshape(-1, 3), vxy.reshape(-1, 2)

    def nodes(self):
        xn = np.zeros(self.Ne * self.np * 2)
        ar = np.zeros(self.Ne)
        lib().pao_get_nodes(self._c, _ptr(xn), _ptr(ar))
        return xn.reshape(self.Ne, self.np, 2), ar

    def ref_tables(self):
        xq = np.zeros(self.nq * 2)
        wq = np.zeros(self.nq)
        ph = np.zeros(self.nq * self.np)
        mh = np.zeros(self.np * self.np)
        lib().pao_ref_tables(self._c, _ptr(xq), _ptr(wq), _ptr(ph), _ptr(mh))
        return xq.reshape(-1, 2), wq, ph.reshape(self.nq, self.np), mh.reshape(self.np, self.np)

    # parameters and fields
    def set_params(self, mu):
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        self._chk(lib().pao_set_params(self._c, _ptr(mu)))

    def gbar(self, n, i):
        out = np.zeros(self.Ne * self.np)
        self._chk(lib().pao_gbar(self._c, n, i, _ptr(out)))
        return out

    def gcl_rhs(self, n, i):
        out = np.zeros(self.Ne * self.np)
        self._chk(lib().pao_gcl_rhs(self._c, n, i, _ptr(out)))
        return out

    def freestream(self, perturb=None):
        u = np.zeros(self.Nu)
        pp = None if perturb is None else self._vec(perturb)
        if lib().pao_freestream(self._c, _ptr(pp), _ptr(u)) != 0:
            raise RuntimeError("freestream before set_params")
        return u

    def mass(self, x):
        x = self._vec(x)
        y = np.zeros(self.Nu)
        lib().pao_mass_apply(self._c, _ptr(x), _ptr(y))
        return y

    def residual(self, n, i, u):
        u = self._vec(u)
        r = np.zeros(self.Nu)
        self._chk(lib().pao_residual(self._c, n, i, _ptr(u), _ptr(r)))
        return r

    def jacobian(self, n, i, u):
        u = self._vec(u)
        blk = np.zeros(self.Ne * 4 * self.b * self.b)
        self._chk(lib().pao_jacobian(self._c, n, i, _ptr(u), _ptr(blk)))
        return blk.reshape(self.Ne, 4, self.b, self.b)

    def dr_dmu(self, n, i, u):
        u = self._vec(u)
        out = np.zeros(3 * self.Nu)
        self._chk(lib().pao_dr_dmu(self._c, n, i, _ptr(u), _ptr(out)))
        return out.reshape(3, self.Nu)

    def qoi(self, n, i, u, derivs=False):
        u = self._vec(u)
        f = np.zeros(2)
        dfdu = np.zeros(2 * self.Nu) if derivs else None
        dfdmu = np.zeros(6) if derivs else None
        self._chk(lib().pao_qoi(self._c, n, i, _ptr(u), _ptr(f), _ptr(dfdu), _ptr(dfdmu)))
        if derivs:
            return f, dfdu.reshape(2, self.Nu), dfdmu.reshape(2, 3)
        return f

    def bsr_apply(self, blk, x, transpose=False):
        blk = np.ascontiguousarray(blk, dtype=np.float64)
        x = self._vec(x)
        y = np.zeros(self.Nu)
        lib().pao_bsr_apply(self._c, _ptr(blk), int(transpose), _ptr(x), _ptr(y))
        return y

    def stage_solve(self, blk, a_dt, rhs, transpose=False):
        blk = np.ascontiguousarray(blk, dtype=np.float64)
        rhs = self._vec(rhs)
        x = np.zeros(self.Nu)
        self._chk(lib().pao_stage_solve(self._c, _ptr(blk), a_dt, int(transpose), _ptr(rhs), _ptr(x)))
        return x

    # sweeps
    def primal_period(self, u0):
        u0 = self._vec(u0)
        uNt = np.zeros(self.Nu)
        q = np.zeros(2)
        res = np.zeros(1)
        self._chk(lib().pao_primal_period(self._c, _ptr(u0), _ptr(uNt), _ptr(q), _ptr(res)))
        return uNt, q, float(res[0])

    def tangent(self, v, mu_dir=-1, with_qoi=False):
        v = self._vec(v)
        out = np.zeros(self.Nu)
        dq = np.zeros(2) if with_qoi else None
        self._chk(lib().pao_tangent_sweep(self._c, _ptr(v), mu_dir, _ptr(out), _ptr(dq)))
        return (out, dq) if with_qoi else out

    def adjoint(self, lamNt, forced_qoi=-1):
        lamNt = self._vec(lamNt)
        out = np.zeros(self.Nu)
        g = np.zeros(3)
        self._chk(lib().pao_adjoint_sweep(self._c, _ptr(lamNt), forced_qoi, _ptr(out), _ptr(g)))
        return (out, g) if forced_qoi >= 0 else out

    def shoot(self, u0, tol=1e-10, eta=1e-6, maxit=30, max_krylov=200):
        u = self._vec(u0).copy()
        rep = pao_krylov_report()
        self._chk(lib().pao_shoot(self._c, _ptr(u), tol, eta, maxit, max_krylov, C.byref(rep)))
        return u, rep

    def periodic_adjoint(self, q, rtol=1e-12, max_krylov=300):
        lam = np.zeros(self.Nu)
        g = np.zeros(3)
        rep = pao_krylov_report()
        self._chk(lib().pao_periodic_adjoint(self._c, q, rtol, max_krylov, _ptr(lam), _ptr(g), C.byref(rep)))
        return g, lam, rep

    def tangent_gradient(self, rtol=1e-12, max_krylov=300):
        dJ = np.zeros(6)
        self._chk(lib().pao_tangent_gradient(self._c, rtol, max_krylov, _ptr(dJ)))
        return dJ.reshape(2, 3)

    def traj(self, which, n, i=1):
        out = np.zeros(self.Nu)
        self._chk(lib().pao_traj(self._c, which, n, i, _ptr(out)))
        return out

    def traj_jacobian(self, n, i):
        blk = np.zeros(self.Ne * 4 * self.b * self.b)
        self._chk(lib().pao_traj_jacobian(self._c, n, i, _ptr(blk)))
        return blk.reshape(self.Ne, 4, self.b, self.b)

    # pointwise fluxes and the face lifting (closed-form pins)
    def flux_vis(self, U, dU, heat=True):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.ascontiguousarray(dU, dtype=np.float64).reshape(8)
        F = np.zeros(8)
        lib().pao_flux_vis(self._c, _ptr(U), _ptr(dU), int(heat), _ptr(F))
        return F.reshape(4, 2)

    def flux_h(self, U, n, vn=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        n = np.ascontiguousarray(n, dtype=np.float64)
        H = np.zeros(4)
        lib().pao_flux_h(self._c, _ptr(U), _ptr(n), float(vn), _ptr(H))
        return H

    def flux_lf(self, UL, UR, n, vn=0.0):
        UL = np.ascontiguousarray(UL, dtype=np.float64)
        UR = np.ascontiguousarray(UR, dtype=np.float64)
        n = np.ascontiguousarray(n, dtype=np.float64)
        F = np.zeros(4)
        lib().pao_flux_lf(self._c, _ptr(UL), _ptr(UR), _ptr(n), float(vn), _ptr(F))
        return F

    def face_lift(self, n, i, u, K, f):
        """(lifting [np][4][2] on the lower-index side, True if that side is K)"""
        u = self._vec(u)
        lift = np.zeros(self.np * 8)
        rc = self._chk(lib().pao_face_lift(self._c, n, i, _ptr(u), K, f, _ptr(lift)))
        return lift.reshape(self.np, 4, 2), rc == 1

    def counters(self):
        a = np.zeros(1, np.int64)
        b = np.zeros(1, np.int64)
        lib().pao_counters(self._c, _ptr(a), _ptr(b))
        return int(a[0]), int(b[0])
