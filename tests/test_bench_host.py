"""Host logic of bench.py, without a GPU: the GPU-count guard, the Section 6
effective-operation count, and the rule that a stored HBM-traffic figure is used
only for the workload and kernel sources it was measured on."""
import os
import subprocess
import sys
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

C2 = dict(workload="n16384_p8388593_r12288_randomrpm", n=16384, p=8388593, r=12288)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


@pytest.mark.parametrize("n", [1, 3, 64, 4096])
def test_effective_ops_full_rank_is_n_cubed_over_3(n):
    # at r = n the count is that of symmetric elimination, n^3/3
    assert bench.eff_ops(n, n) == pytest.approx(n ** 3 / 3.0, rel=1e-15)


def test_effective_ops_terms():
    # r^3/3 + n^2 r - r^2 n, checked in exact rationals on the C2 sizes and at r = 0
    n, r = C2["n"], C2["r"]
    exact = Fraction(r ** 3, 3) + n * n * r - r * r * n
    assert bench.eff_ops(n, r) == pytest.approx(float(exact), rel=1e-15)
    assert bench.eff_ops(n, 0) == 0


@pytest.mark.parametrize("path", ["f64", "i8"])
def test_traffic_figure_bound_to_workload_and_sources(path, tmp_path, monkeypatch):
    got = bench.measured_traffic(path, C2["workload"], C2["n"], C2["p"], C2["r"])
    assert got is not None and got > 0
    # another workload name: not used
    assert bench.measured_traffic(path, "n16384_other", C2["n"], C2["p"], C2["r"]) is None
    # the same sources with one byte changed: not used
    pr = bench.PRODUCT[path]
    for rel in pr["sources"]:
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        with open(os.path.join(ROOT, rel), "rb") as f:
            data = f.read()
        (tmp_path / rel).write_bytes(data + (b" " if rel.endswith(".hip") else b""))
    os.makedirs(tmp_path / "profiles")
    fn = f"{pr['kernel']}.n{C2['n']}_p{C2['p']}_rank{C2['r']}.traffic.txt"
    with open(os.path.join(ROOT, "profiles", fn)) as f:
        (tmp_path / "profiles" / fn).write_text(f.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(path, C2["workload"], C2["n"], C2["p"], C2["r"]) is None
