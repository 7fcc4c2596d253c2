"""Boundary hooks: the context's device memory from the caller's allocator
and its work on the caller's stream (pa_config dev_alloc / dev_free /
stream), with the HIP runtime the library is linked against and with
PyTorch's caching allocator and stream; and the shooting history
(pa_shoot_report res_hist / krylov_hist / step_hist)."""
import ctypes as C
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1512_00616_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KW = dict(Nr=2, Nth=6, p=1, Nt=4, lin_rtol=1e-13, newton_atol=1e-12)


def _run(s):
    s.set_params(np.array(inputs.MU_NOMINAL))
    s.set_freestream(inputs.perturbation(s.Nu, seed=1))
    rep = s.shoot(tol=1e-11, eta=1e-10, maxit=20)
    q, dJ, _ = s.adjoint_gradient(rtol=1e-12)
    return rep, q, dJ, s.get_state(0)


def test_caller_allocator_and_stream():
    """Allocator callbacks (hipMalloc / hipFree of the library's own HIP
    runtime, counted) and a caller-created stream: every device byte of the
    context passes through the callbacks and is returned at destruction, the
    stream is not destroyed by the library, and the results are the bits of
    a default context."""
    from paper_1512_00616_amd import pa
    a = pa.Solver(**KW)
    ra, qa, ga, ua = _run(a)
    a.close()
    hip = C.CDLL("libamdhip64.so.7")     # the runtime already loaded by the library
    live = {}
    AF = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
    FF = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

    def alloc(nbytes, user):
        p = C.c_void_p()
        if hip.hipMalloc(C.byref(p), C.c_size_t(nbytes)) != 0:
            return None
        live[p.value] = nbytes
        return p.value

    def free(ptr, user):
        live.pop(ptr)
        hip.hipFree(C.c_void_p(ptr))

    af, ff = AF(alloc), FF(free)
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    b = pa.Solver(stream=stream.value, dev_alloc=C.cast(af, C.c_void_p).value,
                  dev_free=C.cast(ff, C.c_void_p).value, **KW)
    assert sum(live.values()) == b.device_bytes > 0
    rb, qb, gb, ub = _run(b)
    assert np.array_equal(qa, qb) and np.array_equal(ga, gb) and np.array_equal(ua, ub)
    assert ra.newton_its == rb.newton_its and ra.res == rb.res
    b.close()
    assert live == {}
    assert hip.hipStreamSynchronize(stream) == 0      # still a valid stream
    assert hip.hipStreamDestroy(stream) == 0


_TORCH_CHILD = r"""
import json, sys
import numpy as np
import torch                                   # first: the library then shares torch's HIP runtime
sys.path.insert(0, sys.argv[1])
from paper_1512_00616_amd import pa, inputs
KW = dict(Nr=2, Nth=6, p=1, Nt=4, lin_rtol=1e-13, newton_atol=1e-12)
def run(s):
    s.set_params(np.array(inputs.MU_NOMINAL))
    s.set_freestream(inputs.perturbation(s.Nu, seed=1))
    rep = s.shoot(tol=1e-11, eta=1e-10, maxit=20)
    q, dJ, _ = s.adjoint_gradient(rtol=1e-12)
    return q, dJ, s.get_state(0)
a = pa.Solver(**KW)
qa, ga, ua = run(a)
a.close()
torch.cuda.synchronize()
mem = pa.TorchMemory(device=0)
before = torch.cuda.memory_allocated(0)
b = pa.Solver(memory=mem, **KW)
held0, nb0 = torch.cuda.memory_allocated(0) - before, b.device_bytes    # at creation
qb, gb, ub = run(b)
ev = torch.cuda.Event()
ev.record(mem.stream)
ev.synchronize()
held1, nb1 = torch.cuda.memory_allocated(0) - before, b.device_bytes    # after the lazily sized buffers
b.close()
torch.cuda.synchronize()
after = torch.cuda.memory_allocated(0)
print(json.dumps({"held": [held0, held1], "device_bytes": [nb0, nb1], "returned": after == before,
                  "same_bits": bool(np.array_equal(qa, qb) and np.array_equal(ga, gb) and np.array_equal(ua, ub)),
                  "runtimes": pa.loaded_hip_runtimes()}))
"""


def test_torch_owns_memory_and_stream():
    """PyTorch's caching allocator and a torch stream (in a fresh process
    that imports torch before loading the library, so that both use one HIP
    runtime)."""
    pytest.importorskip("torch")
    r = subprocess.run([sys.executable, "-c", _TORCH_CHILD, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert len(out["runtimes"]) == 1
    for held, nbytes in zip(out["held"], out["device_bytes"]):
        assert held >= nbytes > 0                        # every buffer came from torch's allocator
    assert out["same_bits"]
    assert out["returned"]                               # all of it went back to torch


def test_shooting_history():
    from paper_1512_00616_amd import pa
    s = pa.Solver(**KW)
    rep, *_ = _run(s)
    res, kry, lam = rep.history()
    assert len(res) == rep.newton_its + 1 and res[0] == rep.res0 and res[-1] == rep.res
    assert np.all(np.diff(res) < 0)                  # every accepted step lowers ||R||
    assert kry.sum() == rep.krylov_its and np.all(kry >= 1)
    assert np.all((lam > 0) & (lam <= 1))
    s.close()
