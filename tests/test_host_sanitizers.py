"""The library's host precompute (csrc/host.cpp: Alg. 3, the PSWF solve of App. B, the scaling,
window and residual tables, oversampling, twiddles) built on its own with g++ under the address
and undefined-behaviour sanitizers and run on a set of configurations (tests/host_check.cpp).
Any out-of-bounds access, use after free, leak, signed overflow or other undefined behaviour
aborts the run. Its results must equal what the optimised library returns for the same
arguments (to rounding: the two builds may order floating-point operations differently), and
a few of them are pinned to independent values (Lambert W, the prolate eigenvalue chi_0 from
SciPy, a twiddle factor)."""
import cmath
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

pw = pytest.importorskip("paper_2602_16591_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_16591_amd", "csrc")

# name -> (eps, L, rc, m, n, q_l2, tol_mode, plan precision of the tables); as in host_check.cpp
CASES = {
    "rel_m64": (1e-6, 1.0, 0.0, 64, 0, 0.0, "rel", "fp32"),
    "rel_m30_L1.3": (1e-4, 1.3, 0.0, 30, 0, 0.0, "rel", "fp32"),
    "rel_rc_eps1e-10": (1e-10, 1.0, 0.15, 0, 0, 0.0, "rel", "fp64"),
    "abs_rc": (1e-6, 1.0, 0.15, 0, 0, 10.0, "abs", "fp32"),
    "rel_n5000_L1.5": (1e-6, 1.5, 0.0, 0, 5000, 0.0, "rel", "fp32"),
}


@pytest.fixture(scope="module")
def sanitized_run(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("host_check")
    exe = str(out / "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "host_check.cpp"),
           os.path.join(CSRC, "host.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0 and "ERROR" not in run.stderr and "runtime error" not in run.stderr, \
        run.stderr[-4000:]
    return {r["case"]: r for r in (json.loads(line) for line in run.stdout.splitlines() if line.strip())}


def close(a, b, rel=1e-12):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    assert a.shape == b.shape, (a.shape, b.shape)
    scale = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    assert float(np.max(np.abs(a - b))) <= rel * scale if a.size else True


@pytest.mark.parametrize("name", list(CASES))
def test_sanitized_host_matches_library(sanitized_run, name):
    eps, L, rc, m, n, q_l2, mode, prec = CASES[name]
    r = sanitized_run[name]
    assert r["status"] == 0
    c = pw.choose_params(eps, L, rc=rc, m=m, n=n, q_l2=q_l2, tol_mode=mode)
    assert (r["m"], r["P"]) == (c.m, c.P)
    for k in ("rc", "cs", "cw", "alpha"):
        assert abs(r[k] - getattr(c, k)) <= 1e-13 * abs(getattr(c, k)), k
    t = pw.host_tables(c, prec)
    assert r["deg"] == t["deg"]
    close(np.reshape(r["coef"], (c.P, r["deg"] + 1)), t["coef"], 1e-10)
    close(r["w"], t["w"], 1e-11)
    close(r["tm"], t["tm"], 1e-11)
    assert abs(r["self_coef"] - t["self_coef"]) <= 1e-12 * abs(t["self_coef"])
    o = pw.oversample_params(c, 1.5)
    assert (r["over_status"], r["over_m"], r["over_P"]) == (0, o.m, o.P)


def test_sanitized_cuboid_matches_library(sanitized_run):
    r = sanitized_run["box"]
    assert r["status"] == 0
    c = pw.choose_params_box(1e-6, (1.0, 1.3, 0.8), rc=0.15)
    assert (r["m"], r["my"], r["mz"], r["P"]) == (c.m, c.my, c.mz, c.P)
    assert abs(r["cs"] - c.cs) <= 1e-13 * c.cs


def test_sanitized_host_pinned_values(sanitized_run):
    special = pytest.importorskip("scipy.special")
    r = sanitized_run["misc"]
    assert abs(r["w0_1"] - 0.5671432904097838) < 1e-15            # the omega constant, W0(1)
    assert abs(r["wm1"] - float(special.lambertw(-0.2, -1).real)) < 1e-13
    assert abs(r["chi0_20"] - float(special.pro_cv(0, 0, 20.0))) < 1e-9 * abs(r["chi0_20"])
    z = cmath.exp(2j * cmath.pi * 7 / 60)
    assert r["tw_len"] == 120 and abs(complex(*r["tw_7"]) - z) < 1e-15


def test_sanitizer_build_reports_an_out_of_bounds_read(tmp_path):
    """The same compiler flags on a planted heap overflow: the run must fail with an ASan report,
    so a clean run above means the checks were active."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "oob.cpp"
    src.write_text("#include <vector>\nint main(int argc, char**) { std::vector<int> v(4, 1); "
                   "return v.data()[3 + argc]; }\n")
    exe = str(tmp_path / "oob")
    b = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        str(src), "-o", exe], capture_output=True, text=True, timeout=120)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
