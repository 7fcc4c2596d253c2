"""The allocation-free perceptron pass (pa_mlp_grad_noalloc) against the
allocating one (pa_dbg_mlp) through the C ABI: same kernels on the same
inputs, so the same bits, on two calls in a row (the second smaller, so a
stale entry of the shared work array would show), and a clear error beyond
the work array's size.  Device buffers and the stream come from the HIP
runtime the library is linked against (hipMalloc / hipStreamCreate through
ctypes)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


class _Hip:
    def __init__(self):
        from paper_1512_00616_amd import pa
        pa.lib()                                   # maps the library's HIP runtime first
        self.h = C.CDLL("libamdhip64.so.7")
        self.bufs = []

    def chk(self, rc):
        assert rc == 0, rc

    def to_dev(self, a):
        a = np.ascontiguousarray(a)
        p = C.c_void_p()
        self.chk(self.h.hipMalloc(C.byref(p), C.c_size_t(max(a.nbytes, 4))))
        self.bufs.append(p)
        self.chk(self.h.hipMemcpy(p, a.ctypes.data_as(C.c_void_p), C.c_size_t(a.nbytes), 1))   # host to device
        return p.value

    def to_host(self, ptr, like):
        out = np.empty_like(like)
        self.chk(self.h.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), C.c_size_t(out.nbytes), 2))
        return out

    def close(self):
        for p in self.bufs:
            self.chk(self.h.hipFree(p))
        self.bufs = []


def _case(width, batch, seed, n_in=4, n_out=16):
    g = np.random.default_rng(seed)
    dims = [n_in, width, width, width, n_out]
    parts = []
    for l in range(4):
        a = np.sqrt(6.0 / (dims[l] + dims[l + 1]))
        parts += [g.uniform(-a, a, dims[l + 1] * dims[l]), 0.1 * g.standard_normal(dims[l + 1])]
    p = np.concatenate(parts).astype(np.float32)
    X = g.standard_normal((n_in, batch)).astype(np.float32)
    T = g.standard_normal((n_out, batch)).astype(np.float32)
    return p, X, T


def test_noalloc_pass_matches_allocating_pass_twice():
    from paper_1512_00616_amd import pa
    hip = _Hip()
    stream = C.c_void_p()
    hip.chk(hip.h.hipStreamCreate(C.byref(stream)))
    try:
        for width, batch, seed in ((256, 48, 1), (64, 7, 2)):
            p, X, T = _case(width, batch, seed)
            loss_ref, grads_ref = pa.dbg_mlp(p, X, T, width)
            nan1 = np.full(1, np.nan, np.float32)
            nang = np.full_like(p, np.nan)
            dp, dX, dT, dl, dg = (hip.to_dev(a) for a in (p, X, T, nan1, nang))
            pa.mlp_grad_noalloc(X.shape[0], width, T.shape[0], X.shape[1], dp, dX, dT, dl, dg, stream.value)
            hip.chk(hip.h.hipStreamSynchronize(stream))
            loss = float(hip.to_host(dl, nan1)[0])
            grads = hip.to_host(dg, nang)
            assert loss == loss_ref
            assert np.array_equal(grads, grads_ref)
    finally:
        hip.close()
        hip.chk(hip.h.hipStreamDestroy(stream))


def test_noalloc_rejects_a_pass_beyond_its_work_array():
    from paper_1512_00616_amd import pa
    hip = _Hip()
    width, batch = 256, 1024        # (3*256 + 16 + 2*256) * 1024 floats > 2^20
    p, X, T = _case(width, 4, 3)
    try:
        dp = hip.to_dev(p)
        buf = hip.to_dev(np.zeros(4 * 16 * batch, np.float32))
        with pytest.raises(pa.PaError, match="work memory"):
            pa.mlp_grad_noalloc(4, width, 16, batch, dp, buf, buf, buf, buf, 0)
    finally:
        hip.close()
