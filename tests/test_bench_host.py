"""Host logic of the benchmark (no GPU): the refusal of more than one GPU,
the algorithmic bytes of the outer SpMV counted by hand for the config-3
matrix, and the HBM traffic figure, which is reported only while the SpMV
source it was measured on is unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_spmv_bytes_hand_count():
    # config 3: 1000 x 500 cells, 5-point pattern, b = 8
    n = 1000 * 500
    nnzb = n + 2 * (999 * 500) + 2 * (1000 * 499)
    assert nnzb == 2497000
    values = nnzb * 64 * 8            # FP64 8x8 blocks
    cols = nnzb * 4                   # int32 column indices
    rows = (n + 1) * 4                # int32 row pointers
    vecs = 2 * n * 8 * 8              # x read once, y written once
    assert bench.spmv_algorithmic_bytes(n, nnzb, 8) == values + cols + rows + vecs == 1354452004


def test_traffic_follows_kernel_source(monkeypatch):
    nbytes = bench.spmv_algorithmic_bytes(500000, 2497000, 8)
    t = bench.load_traffic(nbytes)
    assert t is not None and t > nbytes            # measured traffic, above the compulsory bytes
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic(nbytes) is None


def test_traffic_follows_launch_size():
    """The counter summary of one matrix is not reported for another."""
    nbytes = bench.spmv_algorithmic_bytes(500000, 2497000, 8)
    assert bench.load_traffic(nbytes + 8) is None
    assert bench.load_traffic(nbytes, "no_such_summary.json") is None


def test_host_cpu_reports_cores():
    h = bench.host_cpu()
    assert h["nproc"] == os.cpu_count() and h["nproc"] >= 1


def test_cv_across_peclet_hand_worked():
    """CV = population standard deviation / mean: iterations 55, 9, 9 have
    mean 73/3 and deviations 92/3, -46/3, -46/3, so the standard deviation is
    sqrt((92^2 + 2 * 46^2) / 27) = 21.6846 and the CV 0.8911; entries that
    did not converge at every Peclet number are left out."""
    rows = [dict(variant="CPR", subsolves="AMG", grid=64, peclet=pe, iterations=it, converged=1)
            for pe, it in ((0.01, 55), (1.0, 9), (100.0, 9))]
    rows += [dict(variant="X", subsolves="AMG", grid=64, peclet=pe, iterations=10, converged=int(pe != 1.0))
             for pe in (0.01, 1.0, 100.0)]
    cv = bench.cv_across_peclet(rows)
    assert len(cv) == 1 and cv[0]["variant"] == "CPR"
    assert cv[0]["cv"] == 0.8911 and cv[0]["mean"] == 24.333


def test_vcycle_bytes_hand_count():
    """One V-cycle's algorithmic bytes on a two-level hierarchy counted by
    hand: level 0 of 4 rows (10 entries, P with 5), 2 + 2 sweeps in FP32,
    then the dense 2 x 2 inverse of the coarsest level in FP64."""
    class Fake:
        def amg_levels(self, which):
            return 2

        def amg_level_sizes(self, which, level):
            return [(4, 10, 5), (2, 4, 0)][level]

    a_pass = 5 * 4 + 10 * 8
    level0 = ((a_pass + 4 * 4 * 4) + (a_pass + 6 * 4 * 4) + (3 * 4 + 5 * 8 + 4 * 4 + 2 * 4)
              + (5 * 4 + 5 * 8 + 2 * 4 + 2 * 4 * 4) + 2 * (a_pass + 4 * 4 * 4))
    assert level0 == 864
    assert bench.vcycle_bytes(Fake(), 0, 2, 2) == 864 + 2 * 2 * 8 + 2 * 2 * 4
    # the fine level's four sweeps on five planes: 5 x 4 rows x 4 bytes
    # instead of 5 row pointers and 10 (index, value) pairs per pass
    planes = 864 - 4 * a_pass + 4 * (5 * 4 * 4)
    assert bench.vcycle_bytes(Fake(), 0, 2, 2, fine_planes=True) == planes + 2 * 2 * 8 + 2 * 2 * 4
