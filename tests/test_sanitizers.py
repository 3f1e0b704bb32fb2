"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code: the
oracle, the scene generator and the library's host layer (argument checks,
workspace sizing, plans, the JSON tuning-cache reader), driven by
tests/sanitize_driver.cpp. CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe, *args):
    # The OpenMP runtime keeps one internal block until exit; only that library is exempt from leak checks.
    supp = os.path.join(os.path.dirname(exe), "lsan.supp")
    with open(supp, "w") as fh:
        fh.write("leak:libomp.so\nleak:libgomp.so\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               LSAN_OPTIONS=f"suppressions={supp}", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitize driver ok" in r.stdout


def test_oracle_and_scenes_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "drv")
    cmd = ["g++", "-std=c++17", "-fopenmp", *SAN, os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
           os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(ROOT, "scenes", "scenes.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    _run(exe)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not available")
def test_library_host_layer_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "drv_lib")
    csrc = os.path.join(ROOT, "paper_2001_07809_amd", "csrc")
    san_host = []
    for flag in SAN:
        san_host += ["-Xarch_host", flag] if flag.startswith("-fsanitize") else [flag]
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++17", "-fopenmp", *san_host, "-DWITH_LIB",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(ROOT, "tests", "sanitize_driver.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp"),
           os.path.join(ROOT, "scenes", "scenes.cpp"), os.path.join(csrc, "sbs_api.hip"),
           os.path.join(csrc, "sbs_kernels.hip"), os.path.join(csrc, "sbs_post.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    cache = tmp_path / "tuning.json"
    cache.write_text('{\n  "gfx950/96x64x3/b7/d15/rho4": {"cols_per_lane": 4, "chunk": 8, "tile_rows": 32, '
                     '"waves_per_cu": 8},\n  "junk": 3\n}\n')
    _run(exe, str(cache))
