"""Host-side pieces of bench.py: the one-GPU guard, the algorithmic work behind the roofline
figures, and the rule that counter summaries count only for the kernel sources they were taken
on. No GPU is used."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("extra", [[], ["--workload", "uniform_n1e6"]])
def test_more_than_one_gpu_is_refused_with_a_message(extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *extra], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_water_box_counter_summaries_are_not_used_for_other_workloads(tmp_path, monkeypatch):
    blob = {"kernel_source_sha256": bench.kernel_source_sha256(), "workload": "water_box_n30000",
            "bytes_per_launch": {"k_spread_mfma<float, 13, 11, 8, float, false>": 41_000_000, "k_spread_mfma<float, 13, 11, 8, double, false>": 52_000_000}}
    p = tmp_path / "summary.md"
    p.write_text("```json\n" + json.dumps(blob) + "\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    monkeypatch.setattr(bench, "TRAFFIC_FILE_N1E6", str(p))   # a water-box summary where the n = 1e6 one belongs
    assert bench.measured_traffic("spread", "fp32_arith") == 41_000_000
    assert bench.measured_traffic("spread", "fp32") == 52_000_000
    assert bench.measured_traffic("spread", "fp64") is None
    assert bench.measured_traffic("spread", "fp32_arith", "uniform_n1e6") is None


def test_spread_and_gather_work_per_launch():
    # water box: n = 30,000, P = 13, deg = 9
    n, P, deg = 30000, 13, 9
    kind, flops = bench.stage_work("spread", n, 64, P, deg, 4)
    assert kind == "mfma"
    assert flops == n * (3 * P * 2 * deg + 2 * P * P + 2 * P ** 3) == 163_020_000
    kind, flops = bench.stage_work("gather", n, 64, P, deg, 4)
    assert kind == "alu"
    assert flops == n * (6 * P * 2 * deg + 4 * P ** 3 + 6 * P * P + 8 * P)


@pytest.mark.parametrize("elem", [4, 8])
def test_fft_pass_bytes(elem):
    m = 64
    real, half = m ** 3 * elem, m * m * (m // 2 + 1) * 2 * elem
    assert bench.stage_work("fft_x", 1, m, 13, 9, elem) == ("hbm", real + half)
    assert bench.stage_work("ifft_x", 1, m, 13, 9, elem) == ("hbm", half + real)
    for st in ("fft_y", "fft_z_scale", "ifft_y"):
        assert bench.stage_work(st, 1, m, 13, 9, elem) == ("hbm", 2 * half)


def _summary(tmp_path, sha):
    blob = {"kernel_source_sha256": sha, "bytes_per_launch": {"k_spread_mfma<float, 13, 11, 8, float, false>": 41_000_000, "k_spread_mfma<float, 13, 11, 8, double, false>": 52_000_000}}
    p = tmp_path / "summary.md"
    p.write_text("# summary\n\n```json\n" + json.dumps(blob) + "\n```\n")
    return str(p)


def test_counter_summaries_apply_only_to_their_kernel_sources(tmp_path, monkeypatch):
    current = bench.kernel_source_sha256()
    assert len(current) == 64
    assert bench._profile_blob(_summary(tmp_path, current)) is not None
    assert bench._profile_blob(_summary(tmp_path, "0" * 64)) is None
    assert bench._profile_blob(str(tmp_path / "missing.md")) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, current))
    assert bench.measured_traffic("spread", "fp32_arith") == 41_000_000
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, "0" * 64))
    assert bench.measured_traffic("spread", "fp32_arith") is None


def test_roofline_fractions_are_fractions():
    stage_ms = {st: 0.05 for st in bench.STAGES}
    rows = bench.kernel_rooflines(stage_ms, 30000, 64, 13, 9, 4, "fp32_arith")
    for st, row in rows.items():
        frac = row.get("frac_peak", row.get("frac_hbm_peak"))
        assert frac is not None and 0.0 < frac < 1.0, (st, row)


def test_kernel_hash_ignores_comments_but_not_code():
    src = 'int f(int a) {  // twice\n  /* returns\n     double */ return 2 * a; }\nconst char* s = "// kept";\n'
    same = 'int f(int a) { return 2 * a; } // reworded\nconst char* s = "// kept";'
    other = 'int f(int a) { return 3 * a; }\nconst char* s = "// kept";'
    assert bench.code_only(src) == bench.code_only(same)
    assert bench.code_only(src) != bench.code_only(other)
    assert '"// kept"' in bench.code_only(src)


def test_binning_traffic_sums_the_sort_kernels_of_either_form(tmp_path, monkeypatch):
    """The binning stage is three launches: count, scan, scatter (one-level sort) or count,
    coarse pass, fine pass (two-level sort); its traffic is their sum, per storage type."""
    one = {"k_bin_count1<float>": 1, "k_scan": 2, "k_bin_scatter1<float>": 4, "k_bin_count1<double>": 100}
    two = {"k_bin_count<float>": 10, "k_bin_coarse<float>": 20, "k_bin_fine<float>": 40, "k_scan": 1000}
    for per, want, workload in ((one, 7, "water_box_n30000"), (two, 70, "uniform_n1e6")):
        blob = {"kernel_source_sha256": bench.kernel_source_sha256(), "workload": workload, "bytes_per_launch": per}
        p = tmp_path / f"{workload}.md"
        p.write_text("```json\n" + json.dumps(blob) + "\n```\n")
        monkeypatch.setattr(bench, "TRAFFIC_FILE_N1E6" if workload == "uniform_n1e6" else "TRAFFIC_FILE", str(p))
        assert bench.measured_traffic("bin", "fp32_arith", workload) == want
