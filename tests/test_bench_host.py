"""Host-side arithmetic of bench.py (no GPU): the algorithmic bytes of the
stage-operator applies that the roofline divides by the measured launch
time, checked against the block count of the mesh itself, and the
bandwidth of a roofline entry."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    had = os.environ.get("PA_VERBOSE")
    import bench as b        # sets PA_VERBOSE for its own runs: undo that here
    if had is None:
        os.environ.pop("PA_VERBOSE", None)
    return b


@pytest.mark.parametrize("Nr,Nth,p", [(32, 96, 3), (8, 24, 1), (16, 48, 2)])
def test_apply_bytes_count_every_stored_off_diagonal_block(bench, oracle_mod, Nr, Nth, p):
    # the preconditioned operator's diagonal blocks are the identity and are
    # never read: one apply streams one b x b block per element face with a
    # neighbour, plus x and y once per right-hand side
    o = oracle_mod.Oracle(Nr=Nr, Nth=Nth, p=p, Nt=1)
    _, en, _, _ = o.mesh()
    o.close()
    b = 4 * (p + 1) * (p + 2) // 2
    blocks = int((en >= 0).sum())
    Nu = en.shape[0] * b
    for nrhs in (1, 2, 3):
        assert bench.spmv_bytes(Nr, Nth, p, nrhs=nrhs) == blocks * b * b * 8 + nrhs * 2 * Nu * 8
    # FP32 / BF16 operator copies with FP32 vectors
    assert bench.spmv_bytes(Nr, Nth, p, 4, 4) == blocks * b * b * 4 + 2 * Nu * 4
    assert bench.spmv_bytes(Nr, Nth, p, 2, 4) == blocks * b * b * 2 + 2 * Nu * 4


def test_full_size_apply_bytes(bench):
    # 32x96 p=3: 18,240 off-diagonal 40x40 blocks (233.47 MB) + x and y (3.93 MB)
    assert bench.spmv_bytes(32, 96, 3) == 233_472_000 + 3_932_160
    assert bench.spmv_bytes(32, 96, 3, nrhs=2) == 233_472_000 + 2 * 3_932_160


def test_roofline_entry_counts_only_working_launches(bench):
    # 10 launches, 2 of which returned at once: the 8 ms total is spread over
    # the 8 working launches (1 ms each); 8 GB per launch is then 8 TB/s
    e = bench.roofline_entry("k", 8.0, 10, 2, 8e9)
    assert e["avg_launch_us"] == pytest.approx(1000.0)
    assert e["achieved_gbs"] == pytest.approx(8000.0)
    assert e["frac"] == pytest.approx(8000.0 / bench.HBM_PEAK_GBS)
    assert e["avg_launch_us_all"] == pytest.approx(800.0)
    assert bench.roofline_entry("k", 8.0, 4, 4, 8e9) is None
    assert bench.roofline_entry("k", 0.0, 4, 0, 8e9) is None
