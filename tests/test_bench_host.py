"""Host logic of bench.py: the kernel digest that keys counter summaries, the
summary reader, the issue fraction and the one-GPU guard (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_digest_ignores_comments_and_blank_lines(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int a; // one\n\n/* block\n comment */ int b;\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    d0 = bench.kernel_code_digest()
    src.write_text("int a; // another comment\n/* x */ int b;\n\n\n")
    assert bench.kernel_code_digest() == d0
    src.write_text("int a; int b;\n")
    assert bench.kernel_code_digest() != d0


def _profile(dirpath, name, digest, field, value):
    (dirpath / name).write_text(f"# summary\n\n| a | b |\n\nkernel_code_sha256: {digest}\n{field}: {value}\n")


def test_summary_figures_only_for_the_current_kernel(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    cur = bench.kernel_code_digest()
    _profile(tmp_path, "k_w_traffic.md", cur, "traffic_bytes_per_launch", "1234")
    _profile(tmp_path, "old_traffic.md", "0" * 64, "traffic_bytes_per_launch", "99")
    assert bench.measured_traffic("k_w_traffic.md") == 1234
    assert bench.measured_traffic("old_traffic.md") is None
    assert bench.measured_traffic("missing.md") is None
    assert bench.profile_field("k_w_traffic.md", "no_such_field") is None


def test_issue_fraction(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    _profile(tmp_path, "kern_wl_sq_counters.md", bench.kernel_code_digest(), "instructions_per_step", "250.0")
    probes = {"simds": 1024, "clock_khz": 2400000, "mixed_instr_per_s": 1.0e12, "salu_instr_per_s": 6.0e11,
              "dependent_instr_per_s": 8.0e11, "dependent4_instr_per_s": 5.0e11}
    r = bench.issue_fraction(2.0e9, "kern", "wl", probes)
    assert r["achieved"] == pytest.approx(5.0e11)
    assert r["frac_mixed"] == pytest.approx(0.5) and r["frac_dependent"] == pytest.approx(0.625)
    assert r["per_simd_cycle"] == pytest.approx(5.0e11 / (1024 * 2.4e9))
    assert bench.issue_fraction(2.0e9, "kern", "other", probes) is None
    assert bench.issue_fraction(2.0e9, "kern", "wl", None) is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert out.returncode != 0
    assert "one GPU only" in out.stdout + out.stderr
