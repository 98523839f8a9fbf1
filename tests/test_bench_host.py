"""Host-side logic of bench.py (no GPU): the roofline's `traffic` is read from a committed counter
summary only while the kernel sources it was measured on are unchanged."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _summary(path, digest, total):
    path.write_text(
        "# HBM traffic per launch\n\n| kernel | dispatches | HBM read GB | HBM write GB |\n"
        "|---|---:|---:|---:|\n\nMachine-read lines:\n\n"
        "kernel: hmx::aca_kernel<double2, 512, true, 1024>\n"
        f"aca sources sha256[:16]: {digest}\n"
        "hbm_read_bytes_per_launch: 1.0e+11\n"
        "hbm_write_bytes_per_launch: 1.0e+10\n"
        f"hbm_bytes_per_launch: {total:.6e}\n")


def test_traffic_read_while_source_unchanged(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    hdr = tmp_path / "k.h"
    hdr.write_text("kernel header\n")
    summ = tmp_path / "summary.txt"
    _summary(summ, bench.source_digest(str(src), str(hdr)), 1.25e11)
    monkeypatch.setattr(bench, "ACA_SOURCES", (str(src), str(hdr)))
    monkeypatch.setitem(bench.PMC_SUMMARY, "fp64", str(summ))
    assert bench.measured_traffic("fp64") == pytest.approx(1.25e11)


def test_traffic_null_once_source_changes(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    summ = tmp_path / "summary.txt"
    _summary(summ, bench.source_digest(str(src)), 1.25e11)
    src.write_text("kernel source, edited\n")
    monkeypatch.setattr(bench, "ACA_SOURCES", (str(src),))
    monkeypatch.setitem(bench.PMC_SUMMARY, "fp64", str(summ))
    assert bench.measured_traffic("fp64") is None


def test_traffic_null_once_a_header_changes(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    hdr = tmp_path / "k.h"
    hdr.write_text("kernel header\n")
    summ = tmp_path / "summary.txt"
    _summary(summ, bench.source_digest(str(src), str(hdr)), 1.25e11)
    hdr.write_text("kernel header, edited\n")
    monkeypatch.setattr(bench, "ACA_SOURCES", (str(src), str(hdr)))
    monkeypatch.setitem(bench.PMC_SUMMARY, "fp64", str(summ))
    assert bench.measured_traffic("fp64") is None


def test_traffic_null_without_summary(bench, tmp_path, monkeypatch):
    monkeypatch.setitem(bench.PMC_SUMMARY, "fp64", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("fp64") is None


def test_gpus_above_one_refused(bench, monkeypatch, capsys):
    # one GPU per box: the bench says so and exits instead of measuring
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code != 0
