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
