"""Host-side logic of bench.py (no GPU): the refusal of several GPUs, the algorithmic
byte count and the rule that stored counter traffic is used only for the kernel it was
measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_algorithmic_bytes_per_sample():
    # C2: two orders x 2 (read + write) x 7 rows x 128 x 4 B, one edge record, 5 negative records
    assert bench.algorithmic_bytes_per_sample(128, 5, 3, 4) == 2 * 2 * 7 * 512 + 32 + 80
    assert bench.algorithmic_bytes_per_sample(128, 5, 2, 2) == 2 * 7 * 256 + 32 + 80


def _summary(tmp_path, sha, cfg="32 4 16", T=200000000):
    p = tmp_path / "s.md"
    p.write_text("# x\n\n    traffic_bytes_per_launch: 123456\n"
                 f"    kernel_config: {cfg}\n    total_samples: {T}\n    kernel_sources_sha256: {sha}\n")
    return str(p)


def test_traffic_only_for_the_measured_kernel(tmp_path):
    cfg = {"lanes_per_sample": 32, "units_per_lane": 4, "blocks_per_cu": 16}
    sha = bench.kernel_sources_sha256()
    assert bench.measured_traffic(_summary(tmp_path, sha), cfg, 200000000) == 123456.0
    assert bench.measured_traffic(_summary(tmp_path, "0" * 64), cfg, 200000000) is None
    assert bench.measured_traffic(_summary(tmp_path, sha, cfg="16 4 16"), cfg, 200000000) is None
    assert bench.measured_traffic(_summary(tmp_path, sha, T=5), cfg, 200000000) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), cfg, 200000000) is None


def test_committed_traffic_summary_is_parseable():
    rec = {}
    for line in open(bench.TRAFFIC_PROFILE):
        k, sep, v = line.strip().partition(": ")
        if sep:
            rec[k] = v
    assert float(rec["traffic_bytes_per_launch"]) > 0 and len(rec["kernel_sources_sha256"]) == 64


def test_traffic_hash_ignores_comments_only():
    code = 'int a = 1; // note\n/* block\n comment */ const char *s = "// kept";\n'
    assert bench._code_only(code, False) == bench._code_only(code.replace("note", "other"), False)
    assert bench._code_only(code, False) != bench._code_only(code.replace("a = 1", "a = 2"), False)
    assert "// kept" in bench._code_only(code, False)
