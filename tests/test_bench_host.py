"""Host-side parts of bench.py that need no GPU: the one-GPU contract and the
stored hardware-counter traffic, which is reported only while the kernel
sources are the ones the counters were taken on."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""  # no JSON line for a configuration that was not measured


def test_kernel_sources_exist(bench):
    for f in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, f)), f
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()


def test_stored_traffic_follows_the_source_hash(bench, monkeypatch, tmp_path):
    summary = tmp_path / "traffic.txt"
    summary.write_text("# comment: not a key\n"
                       f"source_hash: {bench.kernel_source_hash()}\n"
                       "fetch_scale: 2.0\n"
                       "traffic_bytes[cgs_update]: 120000000\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench.stored_traffic("cgs_update") == 120000000.0
    assert bench.stored_traffic("matvec_dots") is None  # not measured
    # counters taken on other kernel sources are not reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.stored_traffic("cgs_update") is None
    # no summary at all
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.stored_traffic("cgs_update") is None

