"""CPU tests of bench.py's host-side helpers: the time-to-gap beta schedule, the cluster-size
mix of the interval chains' CPU sample, the source-hash gate of the stored traffic figures, and
the single-GPU guard.  Nothing here touches a GPU."""
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_gap_stages_double_beta_then_hold():
    st = bench.gap_stages(12288.0, 500)
    betas = [b for b, _ in st]
    assert betas[0] == 1.0 and betas[-1] == 12288.0
    # doubling while below the final value (1 .. 8192: 14 stages of 500), then open-ended
    assert betas[:-1] == [2.0 ** k for k in range(14)]
    assert all(K == 500 for _, K in st[:-1]) and st[-1][1] is None
    assert bench.gap_stages(1.0, 7) == [(1.0, None)]
    # iterations until beta reaches its final value: the 7000 of the pre-phase
    assert sum(K for _, K in st[:-1]) == 7000


def test_schedule_iter_walks_every_stage_in_order():
    got = list(bench.schedule_iter([(1.0, 2), (2.0, 3)]))
    assert got == [(0, 1.0), (0, 1.0), (1, 2.0), (1, 2.0), (1, 2.0)]


def test_interval_chain_cluster_mix():
    # Y_k on n sites: n - m + 1 intervals of m sites for m = 1..k, against n - k + 1 tops
    assert bench.c3_mix(4096, 8) == pytest.approx(32740 / 4089)
    assert bench.c3_mix(24, 8) == pytest.approx(164 / 17)
    assert bench.c3_mix(100, 1) == 1.0
    # the CPU sample's mix stays within 3 % of the full chain's for every k the bench runs
    for k in range(2, 9):
        assert abs(bench.c3_mix(bench.C3_CPU_SITES, k) / bench.c3_mix(4096, k) - 1) < 0.03


def test_traffic_figures_only_for_the_sources_they_were_measured_on(monkeypatch):
    h = bench.kernel_sources_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.kernel_sources_hash() == h          # deterministic
    rec = dict(bench.TRAFFIC_BYTES)
    monkeypatch.setattr(bench, "TRAFFIC_BYTES", {"c4": ("0" * 16, 123), "c2": (h, 456)})
    assert bench.traffic_bytes("c4") is None          # measured on other sources: reported as null
    assert bench.traffic_bytes("c2") == 456
    assert bench.traffic_bytes("c9") is None
    assert all(len(v[0]) == 16 and v[1] > 0 for v in rec.values())


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, f"{ROOT}/bench.py", "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
