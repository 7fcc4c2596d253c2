"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "pa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    from paper_1512_00616_amd import pa
    assert sorted(pa.EXPORTED) == header_symbols()


def test_library_exports_every_declared_symbol():
    from paper_1512_00616_amd import pa
    lib = ctypes.CDLL(pa.LIB_PATH)
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_oracle_library_exports_its_header():
    src = open(os.path.join(ROOT, "oracle", "oracle.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    syms = sorted(set(re.findall(r"\b(pao_[a-z_0-9]+)\s*\(", src)))
    lib = ctypes.CDLL(os.path.join(ROOT, "oracle", "liboracle.so"))
    assert [s for s in syms if not hasattr(lib, s)] == []


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    # no CPU fallback: with libpa.so absent every call raises
    from paper_1512_00616_amd import pa
    monkeypatch.setattr(pa, "LIB_PATH", str(tmp_path / "libpa.so"))
    monkeypatch.setattr(pa, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError, match="HIP library not built"):
        pa.lib()
    with pytest.raises(RuntimeError, match="HIP library not built"):
        pa.Solver(Nr=2, Nth=6, p=1, Nt=2)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_create_rejects_configurations_before_touching_the_device():
    # pa_create validates the configuration first (no device call), so the
    # refusals below hold without a GPU
    import pytest
    from paper_1512_00616_amd import pa
    base = dict(Nr=2, Nth=6, p=1, Nt=2)
    for bad in (dict(graph=1, gmres_restart=32),          # a graph covers the 5 iterations between checks
                dict(graph=1, precision=pa.PREC_FP32),    # FP64 stage solves only
                dict(graph=1, wg_solve=1),                # exclusive with the one-workgroup solve
                dict(graph=2), dict(lin_guess=2), dict(wg_solve=2), dict(gmres_restart=65)):
        with pytest.raises(pa.PaError) as e:
            pa.Solver(**dict(base, **bad))
        assert e.value.code == pa.PA_EINVAL, bad
    assert pa.default_config().graph == 0


def test_binding_structs_match_the_header_layout(tmp_path):
    # every struct the binding mirrors has the size and field offsets that
    # the C compiler gives the header's declaration
    import ctypes as C
    import shutil
    import subprocess
    import pytest
    from paper_1512_00616_amd import pa
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [pa.pa_config, pa.pa_shoot_report, pa.pa_adjoint_report, pa.pa_batch_opts, pa.pa_opt_opts,
               pa.pa_opt_report, pa.pa_ws_opts]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pa.h"', 'int main(void) {']
    for S in structs:
        n = S.__name__
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (n, n))
        for f in S._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (n, f[0], n, f[0]))
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for S in structs:
        n = S.__name__
        assert got[(n, "size")] == C.sizeof(S), n
        for f in S._fields_:
            assert got[(n, f[0])] == getattr(S, f[0]).offset, (n, f[0])


def test_binding_checks_array_sizes_before_the_call():
    # the library reads and writes a fixed number of entries through each
    # pointer, so the binding refuses an array of another size before any
    # library call (no context and no device needed)
    import numpy as np
    import pytest
    from paper_1512_00616_amd import pa
    s = pa.Solver.__new__(pa.Solver)
    s._c = None
    s.Nu, s.Ne, s.b = 48, 4, 12
    for call in (lambda: s.set_params([0.25, 0.1]),
                 lambda: s.set_state(np.zeros(47)),
                 lambda: s.set_freestream(np.zeros(49)),
                 lambda: s.ws_predict(np.zeros(4)),
                 lambda: s.tangent_sweep(np.zeros((2, 48))),
                 lambda: s.bsr_apply(np.zeros(4 * 4 * 144 - 1), np.zeros(48)),
                 lambda: s.optimize([0.2, 0.1]),
                 lambda: s.prolong_from(dict(Nr=2, Nth=6, p=1), np.zeros(2 * 2 * 6 * 4 * 3 + 1))):
        with pytest.raises(ValueError, match="expected"):
            call()
    with pytest.raises(ValueError, match="C-contiguous"):
        pa._ptr(np.zeros((4, 4))[:, 0])
    with pytest.raises(ValueError, match="square"):
        pa.dbg_hess_eig(np.zeros((3, 4)))
    with pytest.raises(ValueError, match="square"):
        pa.dbg_sym_eig(np.zeros(9))
    X, T = np.zeros((3, 5), np.float32), np.zeros((16, 5), np.float32)
    with pytest.raises(ValueError, match="params"):
        pa.dbg_mlp(np.zeros(pa.mlp_param_count(3, 32, 16) - 1), X, T, 32)
    with pytest.raises(ValueError, match="batch"):
        pa.dbg_mlp(np.zeros(pa.mlp_param_count(3, 32, 16)), X, T[:, :4], 32)
