"""Python binding of libpa.so (the HIP library).

Argument marshalling only: every step of the method runs in the library's
HIP kernels and its C++ orchestrator.  There is no CPU fallback -- importing
this module without a built ``libpa.so`` raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

PA_OK, PA_EINVAL, PA_ENOMEM, PA_EDEVICE, PA_ENOCONV, PA_ENUMERIC, PA_ESTATE = 0, -1, -2, -3, -4, -5, -6
(PA_K_SPMV, PA_K_PRECOND, PA_K_JACOBIAN, PA_K_RESIDUAL, PA_K_BLOCKINV, PA_K_SPMV_LO, PA_K_SPMV_T, PA_K_SPMV_M,
 PA_K_SPMV_TM, PA_K_MDOT, PA_K_GMUPD) = range(11)
PA_K_COUNT = 11

EXPORTED = [
    "pa_default_config", "pa_create", "pa_destroy", "pa_last_error", "pa_num_dofs", "pa_num_elems",
    "pa_block_size", "pa_device_bytes", "pa_get_mesh", "pa_set_params", "pa_set_state", "pa_set_freestream",
    "pa_get_state", "pa_primal_period", "pa_shoot", "pa_fixed_point", "pa_shoot_descent", "pa_periodicity_gradient", "pa_floquet", "pa_adjoint_gradient", "pa_tangent_gradient", "pa_batch_gradients",
    "pa_ws_train", "pa_ws_predict", "pa_ws_pod", "pa_prolong", "pa_ws_shoot", "pa_ws_save", "pa_ws_load", "pa_dbg_mlp", "pa_mlp_grad_noalloc", "pa_tangent_sweep",
    "pa_adjoint_sweep", "pa_dbg_gbar", "pa_dbg_dgbar", "pa_dbg_residual", "pa_dbg_jacobian", "pa_dbg_dr_dmu",
    "pa_dbg_qoi", "pa_dbg_bsr_apply", "pa_dbg_blockinv", "pa_dbg_stage_solve", "pa_dbg_traj", "pa_dbg_hess_eig", "pa_dbg_sym_eig", "pa_optimize", "pa_dbg_qp3", "pa_set_timing",
    "pa_kernel_time", "pa_kernel_skipped", "pa_kernel_vectors", "pa_bench_spmv", "pa_bench_spmv_m", "pa_bench_spmv_lo", "pa_bench_copy", "pa_tuning",
]


class pa_config(C.Structure):
    _fields_ = [
        ("Nr", C.c_int32), ("Nth", C.c_int32), ("p", C.c_int32), ("Nt", C.c_int32),
        ("r_far", C.c_double), ("stretch", C.c_double),
        ("mach", C.c_double), ("re", C.c_double), ("gamma", C.c_double), ("pr", C.c_double),
        ("T", C.c_double), ("r_blend0", C.c_double), ("r_blend1", C.c_double),
        ("wall_is_farfield", C.c_int32), ("gmres_restart", C.c_int32), ("lin_rtol", C.c_double),
        ("newton_atol", C.c_double), ("newton_maxit", C.c_int32), ("max_krylov", C.c_int32),
        ("device", C.c_int32), ("precision", C.c_int32), ("autotune", C.c_int32), ("block_krylov", C.c_int32),
        ("stream", C.c_void_p), ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("user", C.c_void_p),
        ("wg_solve", C.c_int32), ("lin_guess", C.c_int32), ("graph", C.c_int32),
    ]


PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2


class pa_shoot_report(C.Structure):
    _fields_ = [("newton_its", C.c_int32), ("krylov_its", C.c_int32), ("primal_sweeps", C.c_int32),
                ("stage_newton_its", C.c_int32), ("stage_gmres_its", C.c_int64), ("res0", C.c_double),
                ("res", C.c_double), ("ms", C.c_double), ("res_hist", C.POINTER(C.c_double)),
                ("krylov_hist", C.POINTER(C.c_int32)), ("step_hist", C.POINTER(C.c_double)),
                ("hist_cap", C.c_int32)]

    def attach_history(self, cap):
        """caller-owned history buffers of cap entries (kept alive on the report)"""
        self._res_hist = np.full(cap, np.nan)
        self._krylov_hist = np.full(cap, -1, dtype=np.int32)
        self._step_hist = np.full(cap, np.nan)
        self.res_hist = self._res_hist.ctypes.data_as(C.POINTER(C.c_double))
        self.krylov_hist = self._krylov_hist.ctypes.data_as(C.POINTER(C.c_int32))
        self.step_hist = self._step_hist.ctypes.data_as(C.POINTER(C.c_double))
        self.hist_cap = cap

    def history(self):
        """(||R|| after each Newton step incl. the start, tangent sweeps and
        accepted step of each Newton step)"""
        n = self.newton_its
        return (self._res_hist[:n + 1].copy(), self._krylov_hist[:n].copy(), self._step_hist[:n].copy())


class pa_adjoint_report(C.Structure):
    _fields_ = [("krylov_its", C.c_int32 * 2), ("sweeps", C.c_int32), ("rhs_sweeps", C.c_int32),
                ("stage_gmres_its", C.c_int64),
                ("rel_res", C.c_double * 2), ("ms", C.c_double)]


class pa_batch_opts(C.Structure):
    _fields_ = [("workers", C.c_int32), ("shoot_maxit", C.c_int32), ("shoot_tol", C.c_double),
                ("shoot_eta", C.c_double), ("allow_unconverged", C.c_int32), ("adj_rtol", C.c_double),
                ("keep_going", C.c_int32)]


class pa_opt_opts(C.Structure):
    _fields_ = [("obj", C.c_int32), ("obj_sign", C.c_double), ("con", C.c_int32), ("con_value", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("maxit", C.c_int32), ("tol_kkt", C.c_double),
                ("tol_c", C.c_double), ("trust", C.c_double), ("shoot_tol", C.c_double),
                ("shoot_eta", C.c_double), ("shoot_maxit", C.c_int32), ("adj_rtol", C.c_double)]


class pa_opt_report(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("shoots", C.c_int32), ("gradients", C.c_int32),
                ("newton_its", C.c_int32), ("tangent_sweeps", C.c_int32), ("adjoint_sweeps", C.c_int32),
                ("converged", C.c_int32), ("f", C.c_double), ("c", C.c_double), ("kkt", C.c_double),
                ("lam", C.c_double), ("mu", C.c_double * 3), ("ms", C.c_double),
                ("mu_hist", C.POINTER(C.c_double)), ("f_hist", C.POINTER(C.c_double)),
                ("c_hist", C.POINTER(C.c_double)), ("hist_cap", C.c_int32)]

    def attach_history(self, cap):
        self._mu_hist = np.full((cap, 3), np.nan)
        self._f_hist = np.full(cap, np.nan)
        self._c_hist = np.full(cap, np.nan)
        self.mu_hist = self._mu_hist.ctypes.data_as(C.POINTER(C.c_double))
        self.f_hist = self._f_hist.ctypes.data_as(C.POINTER(C.c_double))
        self.c_hist = self._c_hist.ctypes.data_as(C.POINTER(C.c_double))
        self.hist_cap = cap

    def history(self):
        """(mu, objective, constraint violation) at the start and after each
        iteration"""
        n = min(self.iterations + 1, self.hist_cap)
        return self._mu_hist[:n].copy(), self._f_hist[:n].copy(), self._c_hist[:n].copy()


class pa_ws_opts(C.Structure):
    _fields_ = [("modes", C.c_int32), ("width", C.c_int32), ("epochs", C.c_int32), ("lr", C.c_float),
                ("seed", C.c_uint64)]


class PaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpa error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library not built: %s -- run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pa_default_config.argtypes = [C.POINTER(pa_config)]
        L.pa_create.argtypes = [C.POINTER(pa_config), C.POINTER(C.c_void_p)]
        L.pa_destroy.argtypes = [P]
        L.pa_last_error.argtypes = [P]
        L.pa_last_error.restype = C.c_char_p
        for fn in ("pa_num_dofs", "pa_device_bytes"):
            getattr(L, fn).argtypes = [P]
            getattr(L, fn).restype = C.c_int64
        for fn in ("pa_num_elems", "pa_block_size"):
            getattr(L, fn).argtypes = [P]
            getattr(L, fn).restype = C.c_int32
        sig = {
            "pa_create": None,
            "pa_get_mesh": [P, P, P, P, P],
            "pa_set_params": [P, P],
            "pa_set_state": [P, P, C.c_int64],
            "pa_set_freestream": [P, P],
            "pa_get_state": [P, C.c_int32, P, C.c_int64],
            "pa_primal_period": [P, P, P],
            "pa_shoot": [P, C.c_double, C.c_double, C.c_int32, P],
            "pa_batch_gradients": [P, C.c_int32, P, P, P, P, P, P, P],
            "pa_floquet": [P, C.c_int32, C.c_uint64, P, P, P, P],
            "pa_ws_train": [P, P, P, C.c_int32, P, P],
            "pa_ws_predict": [P, P],
            "pa_ws_pod": [P, C.c_int32, P, P, P, P],
            "pa_prolong": [C.POINTER(pa_config), P, P, P],
            "pa_ws_shoot": [P, C.c_double, C.c_double, C.c_int32, P, P],
            "pa_ws_save": [P, C.c_char_p],
            "pa_ws_load": [P, C.c_char_p],
            "pa_dbg_mlp": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P],
            "pa_mlp_grad_noalloc": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P],
            "pa_fixed_point": [P, C.c_int32, P],
            "pa_shoot_descent": [P, C.c_double, C.c_int32, C.c_int32, P],
            "pa_periodicity_gradient": [P, P, P],
            "pa_adjoint_gradient": [P, C.c_double, P, P, P],
            "pa_tangent_gradient": [P, C.c_double, P, P],
            "pa_tangent_sweep": [P, P, P],
            "pa_adjoint_sweep": [P, P, C.c_int32, P, P],
            "pa_dbg_gbar": [P, C.c_int32, C.c_int32, P],
            "pa_dbg_dgbar": [P, C.c_int32, C.c_int32, P],
            "pa_dbg_residual": [P, C.c_int32, C.c_int32, P, P],
            "pa_dbg_jacobian": [P, C.c_int32, C.c_int32, P, P],
            "pa_dbg_dr_dmu": [P, C.c_int32, C.c_int32, P, P],
            "pa_dbg_qoi": [P, C.c_int32, C.c_int32, P, P, P, P],
            "pa_dbg_bsr_apply": [P, P, C.c_double, C.c_double, C.c_int32, P, P],
            "pa_dbg_blockinv": [P, P, C.c_double, P],
            "pa_dbg_stage_solve": [P, P, C.c_double, C.c_int32, P, P, P],
            "pa_dbg_traj": [P, C.c_int32, C.c_int32, C.c_int32, P],
            "pa_dbg_hess_eig": [C.c_int32, P, P, P],
            "pa_dbg_sym_eig": [C.c_int32, P, P, P],
            "pa_optimize": [P, C.POINTER(pa_opt_opts), P, C.POINTER(pa_opt_report)],
            "pa_dbg_qp3": [P, P, P, C.c_double, P, P, P, P],
            "pa_set_timing": [P, C.c_int32],
            "pa_kernel_time": [P, C.c_int32, P, P],
            "pa_kernel_skipped": [P, C.c_int32, P],
            "pa_kernel_vectors": [P, C.c_int32, P],
            "pa_bench_spmv": [P, C.c_int32, C.c_int32, P],
            "pa_bench_spmv_m": [P, C.c_int32, C.c_int32, C.c_int32, P],
            "pa_bench_spmv_lo": [P, C.c_int32, C.c_int32, P],
            "pa_tuning": [P, P, P],
            "pa_bench_copy": [P, C.c_int32, P, P],
        }
        for fn, args in sig.items():
            f = getattr(L, fn)
            if args is not None:
                f.argtypes = args
            f.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array arguments must be C-contiguous")
    return a.ctypes.data_as(C.c_void_p)


def _sized(a, n, dtype, what):
    """a as a contiguous array of exactly n entries of dtype (the library
    reads and writes that many through the pointer)"""
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.size != n:
        raise ValueError("%s: expected %d entries, got %d" % (what, n, a.size))
    return a


def _square(a, what):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("%s: expected a square matrix, got shape %s" % (what, a.shape))
    return a


def mlp_param_count(n_in, width, n_out):
    """entries of the perceptron's flat parameter vector [W1 b1 .. W4 b4]"""
    return n_in * width + width + 2 * (width * width + width) + width * n_out + n_out


def default_config(**kw):
    cfg = pa_config()
    lib().pa_default_config(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def batch_gradients(mu, workers=4, shoot_maxit=30, shoot_tol=1e-8, shoot_eta=1e-3, allow_unconverged=False,
                    adj_rtol=1e-8, return_states=False, keep_going=False, direct=False, **cfg_kw):
    """Alg. 4 for every row of mu (n x 3) on one configuration, run by
    `workers` concurrent contexts inside the library; returns qoi (n x 2),
    dJ/dmu (n x 2 x 3), the final periodicity residuals (n), with
    return_states the periodic initial states (n x N_u) and with direct the
    direct-method dJ/dmu (n x 2 x 3; three parameter tangents per
    instance besides the two adjoints)."""
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1, 3))
    n = mu.shape[0]
    cfg = default_config(**cfg_kw)
    o = pa_batch_opts(workers, shoot_maxit, shoot_tol, shoot_eta, int(allow_unconverged), adj_rtol, int(keep_going))
    q = np.zeros((n, 2))
    g = np.zeros((n, 6))
    per = np.zeros(n)
    states = None
    if return_states:
        np_ = (cfg.p + 1) * (cfg.p + 2) // 2
        states = np.zeros((n, 2 * cfg.Nr * cfg.Nth * 4 * np_))
    gd = np.zeros((n, 6)) if direct else None
    rc = lib().pa_batch_gradients(C.byref(cfg), n, _ptr(mu), C.byref(o), _ptr(q), _ptr(g), _ptr(per), _ptr(states),
                                  _ptr(gd))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())
    out = (q, g.reshape(n, 2, 3), per)
    if return_states:
        out = out + (states,)
    if direct:
        out = out + (gd.reshape(n, 2, 3),)
    return out


def dbg_mlp(params, X, T, width):
    """One device forward/backward pass of the warm-start perceptron
    (X [in][batch], T [out][batch]); returns (loss, grads)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    T = np.ascontiguousarray(T, dtype=np.float32)
    if X.ndim != 2 or T.ndim != 2 or X.shape[1] != T.shape[1]:
        raise ValueError("X [in][batch] and T [out][batch] need the same batch, got %s and %s" % (X.shape, T.shape))
    params = _sized(params, mlp_param_count(X.shape[0], width, T.shape[0]), np.float32, "params")
    grads = np.zeros_like(params)
    loss = np.zeros(1, dtype=np.float32)
    rc = lib().pa_dbg_mlp(X.shape[0], width, T.shape[0], X.shape[1], _ptr(params), _ptr(X), _ptr(T), _ptr(loss),
                          _ptr(grads))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())
    return float(loss[0]), grads


def dbg_qp3(B, g, a, c, lo, hi):
    """pa_dbg_qp3: (d, lam) of min g.d + d^T B d / 2, a.d = -c, lo <= d <= hi"""
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(9)
    g, a, lo, hi = (np.ascontiguousarray(v, dtype=np.float64).reshape(3) for v in (g, a, lo, hi))
    d = np.zeros(3)
    lam = np.zeros(1)
    rc = lib().pa_dbg_qp3(_ptr(B), _ptr(g), _ptr(a), float(c), _ptr(lo), _ptr(hi), _ptr(d), _ptr(lam))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())
    return d, float(lam[0])


def mlp_grad_noalloc(n_in, width, n_out, batch, params, X, T, loss, grads, stream=0):
    """pa_mlp_grad_noalloc on device pointers (integers, e.g. torch
    tensors' data_ptr()) enqueued on `stream` (integer handle, 0 = null
    stream); nothing is allocated and nothing is waited for."""
    rc = lib().pa_mlp_grad_noalloc(n_in, width, n_out, batch, C.c_void_p(params), C.c_void_p(X), C.c_void_p(T),
                                   C.c_void_p(loss), C.c_void_p(grads), C.c_void_p(stream))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())


def dbg_hess_eig(H):
    """Eigenvalues (complex, by decreasing modulus) of an upper Hessenberg
    matrix by the library's host-side shifted QR (no device work)."""
    H = _square(H, "H")
    n = H.shape[0]
    re = np.zeros(n)
    im = np.zeros(n)
    rc = lib().pa_dbg_hess_eig(n, _ptr(H), _ptr(re), _ptr(im))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())
    return re + 1j * im


def dbg_sym_eig(A):
    """(eigenvalues descending, eigenvectors as columns) of a symmetric
    matrix by the library's host-side cyclic Jacobi (no device work)."""
    A = _square(A, "A")
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    rc = lib().pa_dbg_sym_eig(n, _ptr(A), _ptr(w), _ptr(V))
    if rc != PA_OK:
        raise PaError(rc, lib().pa_last_error(None).decode())
    return w, V


def loaded_hip_runtimes():
    """paths of the HIP runtime libraries mapped into this process"""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                part = line.split()
                if len(part) >= 6 and "libamdhip64" in part[-1]:
                    paths.add(part[-1])
    except OSError:
        pass
    return sorted(paths)


class TorchMemory:
    """PyTorch owns a context's device memory and stream: every device buffer
    comes from torch's caching allocator (pa_config dev_alloc / dev_free)
    and all device work is enqueued on a torch stream (pa_config stream).
    Keep the object alive as long as the context (Solver keeps a reference).

    Streams are objects of one HIP runtime, so the library and torch must
    share it: import torch before this library is loaded (the dynamic
    linker then resolves the library's HIP runtime to the one torch
    loaded).  A process that mapped two different HIP runtimes is refused."""

    def __init__(self, device=0, stream=None):
        import torch
        lib()
        rts = loaded_hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError("PyTorch and libpa use different HIP runtimes (%s); import torch before the "
                               "library is loaded" % ", ".join(rts))
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        AF = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
        FF = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

        def alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=self.stream)
            except RuntimeError:
                return None

        def free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._af, self._ff = AF(alloc), FF(free)

    def apply(self, cfg):
        cfg.stream = self.stream.cuda_stream
        cfg.dev_alloc = C.cast(self._af, C.c_void_p).value
        cfg.dev_free = C.cast(self._ff, C.c_void_p).value
        cfg.user = None


class Solver:
    """One discretised problem on one GPU (a ``pa_ctx``).  memory: a
    TorchMemory to let PyTorch own the device memory and the stream."""

    def __init__(self, memory=None, **kw):
        self.cfg = default_config(**kw)
        self._memory = memory
        if memory is not None:
            memory.apply(self.cfg)
        h = C.c_void_p()
        rc = lib().pa_create(C.byref(self.cfg), C.byref(h))
        if rc != PA_OK:
            raise PaError(rc, lib().pa_last_error(None).decode())
        self._c = h
        self.Nu = lib().pa_num_dofs(h)
        self.Ne = lib().pa_num_elems(h)
        self.b = lib().pa_block_size(h)
        self.np = self.b // 4
        self.Nt = self.cfg.Nt
        self.mach = self.cfg.mach

    def close(self):
        if getattr(self, "_c", None):
            lib().pa_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != PA_OK:
            raise PaError(rc, lib().pa_last_error(self._c).decode())

    def _vec(self, x, n=None):
        return _sized(x, self.Nu if n is None else n, np.float64, "vector")

    @property
    def device_bytes(self):
        return lib().pa_device_bytes(self._c)

    def mesh(self):
        ev = np.zeros(self.Ne * 3, np.int32)
        en = np.zeros(self.Ne * 3, np.int32)
        tw = np.zeros(self.Ne * 3, np.int8)
        vxy = np.zeros((self.cfg.Nr + 1) * self.cfg.Nth * 2)
        self._chk(lib().pa_get_mesh(self._c, _ptr(ev), _ptr(en), _ptr(tw), _ptr(vxy)))
        return ev.reshape(-1, 3), en.reshape(-1, 3), tw.reshape(-1, 3), vxy.reshape(-1, 2)

    def set_params(self, mu):
        self._chk(lib().pa_set_params(self._c, _ptr(self._vec(mu, 3))))

    def set_state(self, u0):
        u0 = self._vec(u0)
        self._chk(lib().pa_set_state(self._c, _ptr(u0), self.Nu))

    def set_freestream(self, perturb=None):
        pp = None if perturb is None else self._vec(perturb)
        self._chk(lib().pa_set_freestream(self._c, _ptr(pp)))

    def get_state(self, which=0):
        out = np.zeros(self.Nu)
        self._chk(lib().pa_get_state(self._c, which, _ptr(out), self.Nu))
        return out

    def primal_period(self):
        q = np.zeros(2)
        r = np.zeros(1)
        self._chk(lib().pa_primal_period(self._c, _ptr(q), _ptr(r)))
        return q, float(r[0])

    def shoot(self, tol=1e-8, eta=1e-3, maxit=30, allow_unconverged=False):
        """Newton-Krylov shooting; with allow_unconverged the report of a run
        that stopped at maxit Newton steps is returned instead of raising."""
        rep = pa_shoot_report()
        rep.attach_history(maxit + 1)
        rc = lib().pa_shoot(self._c, tol, eta, maxit, C.byref(rep))
        if rc == PA_ENOCONV and allow_unconverged and rep.primal_sweeps > 0:
            return rep
        self._chk(rc)
        return rep

    def floquet(self, k=40, seed=13):
        """Ritz values of Phi (complex, by decreasing modulus) and the last
        Arnoldi subdiagonal entry."""
        re = np.zeros(k)
        im = np.zeros(k)
        n = np.zeros(1, dtype=np.int32)
        h = np.zeros(1)
        self._chk(lib().pa_floquet(self._c, k, seed, _ptr(re), _ptr(im), _ptr(n), _ptr(h)))
        return (re + 1j * im)[: n[0]], float(h[0])

    def optimize(self, mu0, obj=0, obj_sign=-1.0, con=1, con_value=0.0, lo=(0.0, 0.0, 0.0),
                 hi=(1.0, 1.0, 1.0), maxit=20, tol_kkt=1e-6, tol_c=1e-8, trust=0.0, shoot_tol=1e-10,
                 shoot_eta=1e-6, shoot_maxit=30, adj_rtol=1e-10):
        """Periodic-constrained optimisation (pa_optimize); returns (mu,
        report) with the report's history attached."""
        o = pa_opt_opts(obj=obj, obj_sign=obj_sign, con=con, con_value=con_value, maxit=maxit,
                        tol_kkt=tol_kkt, tol_c=tol_c, trust=trust, shoot_tol=shoot_tol, shoot_eta=shoot_eta,
                        shoot_maxit=shoot_maxit, adj_rtol=adj_rtol)
        o.lo[:] = [float(v) for v in lo]
        o.hi[:] = [float(v) for v in hi]
        mu = _sized(np.array(mu0, dtype=np.float64), 3, np.float64, "mu0")
        rep = pa_opt_report()
        rep.attach_history(maxit + 1)
        self._chk(lib().pa_optimize(self._c, C.byref(o), _ptr(mu), C.byref(rep)))
        return mu, rep

    def fixed_point(self, periods):
        r = np.zeros(1)
        self._chk(lib().pa_fixed_point(self._c, periods, _ptr(r)))
        return float(r[0])

    def shoot_descent(self, tol=1e-8, memory=5, maxit=200, allow_unconverged=False):
        """Shooting by minimising 1/2 ||u^(Nt) - u0||^2: steepest descent
        (memory 0) or L-BFGS.  Report fields: newton_its = iterations,
        krylov_its = backward sweeps, primal_sweeps, res0, res."""
        rep = pa_shoot_report()
        rc = lib().pa_shoot_descent(self._c, tol, memory, maxit, C.byref(rep))
        if rc == PA_ENOCONV and allow_unconverged and rep.primal_sweeps > 0:
            return rep
        self._chk(rc)
        return rep

    def periodicity_gradient(self):
        """(dj/du0, j) of j = 1/2 ||u^(Nt) - u0||^2 at the stored trajectory"""
        g = np.zeros(self.Nu)
        j = C.c_double()
        self._chk(lib().pa_periodicity_gradient(self._c, _ptr(g), C.byref(j)))
        return g, j.value

    def adjoint_gradient(self, rtol=1e-8):
        q = np.zeros(2)
        g = np.zeros(6)
        rep = pa_adjoint_report()
        self._chk(lib().pa_adjoint_gradient(self._c, rtol, _ptr(q), _ptr(g), C.byref(rep)))
        return q, g.reshape(2, 3), rep

    # learned warm start
    def ws_train(self, params, states, modes=16, width=256, epochs=2000, lr=1e-3, seed=5, mach=None):
        """params [S][4] = (h0, theta0, phi, Mach), or [S][3] with every state
        at `mach` (default: this context's Mach number)"""
        params = np.asarray(params, dtype=np.float64)
        if params.ndim == 2 and params.shape[1] == 3:
            m = self.mach if mach is None else mach
            params = np.concatenate([params, np.full((params.shape[0], 1), m)], axis=1)
        params = np.ascontiguousarray(params.reshape(-1, 4))
        states = np.ascontiguousarray(np.asarray(states, dtype=np.float64).reshape(params.shape[0], self.Nu))
        o = pa_ws_opts(modes, width, epochs, lr, seed)
        loss = np.zeros(1)
        self._chk(lib().pa_ws_train(self._c, _ptr(params), _ptr(states), params.shape[0], C.byref(o), _ptr(loss)))
        return float(loss[0])

    def ws_predict(self, mu):
        self._chk(lib().pa_ws_predict(self._c, _ptr(self._vec(mu, 3))))

    def ws_pod(self, kmax=128):
        """(mean deviation [Nu], modes [k][Nu], Gram eigenvalues [k])"""
        k = np.zeros(1, dtype=np.int32)
        self._chk(lib().pa_ws_pod(self._c, 0, None, None, None, _ptr(k)))
        kk = min(int(k[0]), kmax)
        mean = np.zeros(self.Nu)
        modes = np.zeros((kk, self.Nu))
        eig = np.zeros(kk)
        self._chk(lib().pa_ws_pod(self._c, kk, _ptr(mean), _ptr(modes), _ptr(eig), _ptr(k)))
        return mean, modes, eig

    def prolong_from(self, coarse, u_coarse):
        """a state of the discretisation `coarse` (dict of pa_config fields)
        evaluated at this context's nodes"""
        cfg = default_config(**coarse)
        n_coarse = 2 * cfg.Nr * cfg.Nth * 4 * ((cfg.p + 1) * (cfg.p + 2) // 2)
        u_coarse = _sized(u_coarse, n_coarse, np.float64, "u_coarse")
        out = np.zeros(self.Nu)
        self._chk(lib().pa_prolong(C.byref(cfg), _ptr(u_coarse), self._c, _ptr(out)))
        return out

    def ws_shoot(self, tol=1e-8, eta=1e-3, maxit=30):
        rep = pa_shoot_report()
        rep.attach_history(maxit + 1)
        fb = np.zeros(1, dtype=np.int32)
        self._chk(lib().pa_ws_shoot(self._c, tol, eta, maxit, C.byref(rep), _ptr(fb)))
        return rep, bool(fb[0])

    def ws_save(self, path):
        self._chk(lib().pa_ws_save(self._c, str(path).encode()))

    def ws_load(self, path):
        self._chk(lib().pa_ws_load(self._c, str(path).encode()))

    def tangent_gradient(self, rtol=1e-8):
        """Direct-method dJ/dmu (2 x 3) and the outer Krylov counts per parameter."""
        g = np.zeros(6)
        its = np.zeros(3, dtype=np.int32)
        self._chk(lib().pa_tangent_gradient(self._c, rtol, _ptr(g), _ptr(its)))
        return g.reshape(2, 3), its

    def tangent_sweep(self, v):
        v = self._vec(v)
        out = np.zeros(self.Nu)
        self._chk(lib().pa_tangent_sweep(self._c, _ptr(v), _ptr(out)))
        return out

    def adjoint_sweep(self, lam, forced_qoi=-1):
        lam = self._vec(lam)
        out = np.zeros(self.Nu)
        g = np.zeros(3)
        self._chk(lib().pa_adjoint_sweep(self._c, _ptr(lam), forced_qoi, _ptr(out), _ptr(g)))
        return (out, g) if forced_qoi >= 0 else out

    # unit-level parity entry points
    def gbar(self, n, i):
        out = np.zeros(self.Ne * self.np)
        self._chk(lib().pa_dbg_gbar(self._c, n, i, _ptr(out)))
        return out

    def dgbar(self, n, i):
        out = np.zeros(3 * self.Ne * self.np)
        self._chk(lib().pa_dbg_dgbar(self._c, n, i, _ptr(out)))
        return out.reshape(3, -1)

    def residual(self, n, i, u):
        r = np.zeros(self.Nu)
        self._chk(lib().pa_dbg_residual(self._c, n, i, _ptr(self._vec(u)), _ptr(r)))
        return r

    def jacobian(self, n, i, u):
        blk = np.zeros(self.Ne * 4 * self.b * self.b)
        self._chk(lib().pa_dbg_jacobian(self._c, n, i, _ptr(self._vec(u)), _ptr(blk)))
        return blk.reshape(self.Ne, 4, self.b, self.b)

    def dr_dmu(self, n, i, u):
        out = np.zeros(3 * self.Nu)
        self._chk(lib().pa_dbg_dr_dmu(self._c, n, i, _ptr(self._vec(u)), _ptr(out)))
        return out.reshape(3, self.Nu)

    def qoi(self, n, i, u):
        f = np.zeros(2)
        dfdu = np.zeros(2 * self.Nu)
        dfdmu = np.zeros(6)
        self._chk(lib().pa_dbg_qoi(self._c, n, i, _ptr(self._vec(u)), _ptr(f), _ptr(dfdu), _ptr(dfdmu)))
        return f, dfdu.reshape(2, self.Nu), dfdmu.reshape(2, 3)

    def bsr_apply(self, blk, x, alpha=0.0, beta=1.0, transpose=False):
        blk = self._vec(blk, self.Ne * 4 * self.b * self.b)
        y = np.zeros(self.Nu)
        self._chk(lib().pa_dbg_bsr_apply(self._c, _ptr(blk), alpha, beta, int(transpose), _ptr(self._vec(x)),
                                         _ptr(y)))
        return y

    def blockinv(self, blk, a_dt):
        blk = self._vec(blk, self.Ne * 4 * self.b * self.b)
        out = np.zeros(self.Ne * self.b * self.b)
        self._chk(lib().pa_dbg_blockinv(self._c, _ptr(blk), a_dt, _ptr(out)))
        return out.reshape(self.Ne, self.b, self.b)

    def stage_solve(self, blk, a_dt, rhs, transpose=False):
        blk = self._vec(blk, self.Ne * 4 * self.b * self.b)
        x = np.zeros(self.Nu)
        its = C.c_int32()
        self._chk(lib().pa_dbg_stage_solve(self._c, _ptr(blk), a_dt, int(transpose), _ptr(self._vec(rhs)),
                                           _ptr(x), C.byref(its)))
        return x, its.value

    def traj(self, which, n, i=1):
        out = np.zeros(self.Nu)
        self._chk(lib().pa_dbg_traj(self._c, which, n, i, _ptr(out)))
        return out

    # measurement
    def set_timing(self, on):
        self._chk(lib().pa_set_timing(self._c, int(on)))

    def kernel_time(self, k):
        ms = C.c_double()
        cnt = C.c_int64()
        self._chk(lib().pa_kernel_time(self._c, k, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def kernel_skipped(self, k):
        """launches of kernel k (since set_timing(True)) that returned at once
        because their GMRES systems had already converged"""
        n = C.c_int64()
        self._chk(lib().pa_kernel_skipped(self._c, k, C.byref(n)))
        return n.value

    def kernel_vectors(self, k):
        """length-Nu vectors read or written by the working launches of the
        stage-GMRES vector kernel k (PA_K_MDOT, PA_K_GMUPD) since
        set_timing(True)"""
        n = C.c_int64()
        self._chk(lib().pa_kernel_vectors(self._c, k, C.byref(n)))
        return n.value

    def bench_copy(self, reps=20):
        ms = C.c_double()
        nb = C.c_int64()
        self._chk(lib().pa_bench_copy(self._c, reps, C.byref(ms), C.byref(nb)))
        return ms.value, nb.value

    def bench_spmv(self, reps=50, transpose=False, nrhs=None):
        ms = C.c_double()
        if nrhs is None:
            self._chk(lib().pa_bench_spmv(self._c, reps, int(transpose), C.byref(ms)))
        else:
            self._chk(lib().pa_bench_spmv_m(self._c, reps, int(transpose), int(nrhs), C.byref(ms)))
        return ms.value

    def tuning(self):
        """(chunks per task of the forward apply, [us per launch for 1, 2, 4])"""
        q = np.zeros(1, dtype=np.int32)
        us = np.zeros(3)
        self._chk(lib().pa_tuning(self._c, _ptr(q), _ptr(us)))
        return int(q[0]), us.tolist()

    def bench_spmv_lo(self, reps=50, transpose=False):
        ms = C.c_double()
        self._chk(lib().pa_bench_spmv_lo(self._c, reps, int(transpose), C.byref(ms)))
        return ms.value
