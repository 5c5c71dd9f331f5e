"""bench.py on the host: the one-GPU contract and the counter bookkeeping (no GPU needed)."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_figures_are_keyed_to_the_kernel_code(tmp_path, monkeypatch):
    """Counter figures are read only while the summary names the current kernel code's hash."""
    import bench
    sha = bench.kernel_code_sha256()
    f = tmp_path / "c.md"
    f.write_text(f"# x\n\n`kernel_code_sha256: {sha}`\n`fp32_3m.fetch_bytes: 1.5e10`\n"
                 "`fp32_3m.write_bytes: 2e9`\n`fp32_3m.mfma_busy: 0.85`\nfp32.mfma_busy: 0.9\n")
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(f))
    got = bench.counter_figures("fp32_3m")
    assert got == {"fetch_bytes": 1.5e10, "write_bytes": 2e9, "mfma_busy": 0.85}
    assert bench.counter_figures("fp32") == {"mfma_busy": 0.9}
    assert bench.counter_figures("bf16x3") is None
    f.write_text(f.read_text().replace(sha, "0" * 64))
    assert bench.counter_figures("fp32_3m") is None          # stale: another kernel
    monkeypatch.setattr(bench, "COUNTER_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.counter_figures("fp32_3m") is None


def test_kernel_code_hash_ignores_comments_only(tmp_path):
    """The key changes with the code and not with comments or blank lines."""
    import bench
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {  // doubled\n  return 2 * x;\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("// a note\nint f(int x) {   // twice x\n\n  return 2 * x;\n}\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) {\n  return 3 * x;\n}\n")
    assert bench.kernel_code_sha256(str(a)) == bench.kernel_code_sha256(str(b))
    assert bench.kernel_code_sha256(str(a)) != bench.kernel_code_sha256(str(c))


def test_level_errors_definition():
    """Per level: max error over the reference's peak, rms error over the reference's rms; empty levels skipped."""
    import bench
    want = np.array([[1.0, -2.0, 4.0], [0.0, 0.0, 0.0], [3.0, 3.0, 3.0]])
    got = want + np.array([[0.4, 0.0, 0.0], [5.0, 0.0, 0.0], [0.0, 0.0, -0.3]])
    mx, rms = bench.level_errors(got, want)
    assert np.allclose(mx, [0.1, 0.1])
    assert np.allclose(rms, [np.sqrt(0.16 / 3 / (21 / 3)), np.sqrt(0.09 / 3 / 9.0)])
