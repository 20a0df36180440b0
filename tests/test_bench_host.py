"""Host-side arithmetic of bench.py's oracle baselines (no GPU)."""
import math

import pytest

import bench


def test_mix_cpu_baseline_is_cores_over_mean_galaxy_time():
    orc = {"s_per_eval": {25: 1e-3, 41: 2e-3}, "cores": 4, "evals": 10, "wall": 1.0, "sample": "s"}
    cb = bench.mix_cpu_baseline(orc, {25: 1, 41: 3}, {25: 100, 41: 100}, "n")
    # mean seconds per galaxy = (1 x 0.1 + 3 x 0.2) / 4 = 0.175
    assert cb["value"] == pytest.approx(4 / 0.175, rel=1e-6)
    assert cb["s_per_galaxy_by_size"] == {25: 0.1, 41: 0.2}
    assert cb["kind"] == "oracle" and cb["cores"] == 4


@pytest.mark.parametrize("name,size,expect_n", [("tiny", None, 32), ("uneven", 41, 41)])
def test_oracle_chain_counts_its_evaluations(name, size, expect_n):
    N, sec, evals = bench._oracle_chain((name, 0, 2, 1, size))
    assert N == expect_n
    assert evals == 3 * bench.gen.CONFIGS[name].leapfrog
    assert math.isfinite(sec) and sec > 0
