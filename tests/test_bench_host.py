"""Host-side checks of the benchmark's measurement code (no GPU): the algorithmic-byte
formulas against hand counts, the counter-summary lookup (current sources only), and
the single-GPU contract of the command line."""
from __future__ import annotations

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_by_hand():
    # one tet, four nodes, 10 pairs, 10 entries, FP32
    b = bench.algorithmic_bytes(4, 1, 4, 10, "fp32")
    assert b["count"] == 16                                  # connectivity
    assert b["integrate"] == 16 + 8 + 24 * 4 + (6 + 4) * 10   # E, c, C in; (row16, col, value) out
    assert b["histogram"] == 2 * 10
    assert b["partition"] == 10 * 10 + 8 * 10
    assert b["reduce"] == 8 * 10 + 8 * 10 + 4 * 4
    assert b["compress"] == 2 * 8 * 10 + 8 * 4
    assert b["path"] == 16 + 8 + 96 + 2 * 4 * 10 + 8 * 10 + 4 * 5
    # FP64 values are 8 bytes wherever a value moves
    b64 = bench.algorithmic_bytes(4, 1, 4, 10, "fp64")
    assert b64["integrate"] - b["integrate"] == 4 * 10
    assert b64["path"] - b["path"] == 2 * 4 * 10 + 4 * 10


def test_stored_traffic_needs_current_sources(tmp_path, monkeypatch):
    summary = tmp_path / "counters_cX_fp32fb64.md"
    summary.write_text(f"# t\nsource_sha256: {bench.source_digest()}\n\n## k_a\ntraffic_bytes: 123\n\n"
                       "## k_a_b\ntraffic_bytes: 456\n")
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    assert bench.stored_traffic("k_a", "cX", "fp32fb64") == 123.0
    assert bench.stored_traffic("k_a_b", "cX", "fp32fb64") == 456.0  # exact section names
    assert bench.stored_traffic("k_c", "cX", "fp32fb64") is None
    summary.write_text("# t\nsource_sha256: 0000\n\n## k_a\ntraffic_bytes: 123\n")
    assert bench.stored_traffic("k_a", "cX", "fp32fb64") is None  # counters of other sources


def test_committed_counter_summaries_name_their_sources():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("counters_"):
            text = open(os.path.join(ROOT, "profiles", name)).read()
            assert "source_sha256:" in text and "rocprofv3 --pmc" in text, name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_pass1_kernel_names_the_launched_variant():
    """The roofline's pass-1 kernel is the one the launch code picks (and a name that
    occurs in the kernel sources)."""
    src = open(os.path.join(os.path.dirname(bench.__file__), "paper_1501_04784_amd", "csrc", "kb_assemble.hpp")).read()
    cases = {(4, "fp32fb64", "stiffness"): "k_pass1_tet", (4, "fp64", "mass"): "k_pass1_tet",
             (8, "fp64", "stiffness"): "k_pass1_two", (8, "fp64", "mass"): "k_pass1_two",
             (8, "fp32fb64", "stiffness"): "k_pass1_pair", (8, "fp32", "mass"): "k_pass1"}
    for (elem, prec, op), name in cases.items():
        assert bench.pass1_kernel(elem, prec, op) == name
        assert f"void {name}(" in src
