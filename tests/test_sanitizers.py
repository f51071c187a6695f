"""The oracle and the host build of the kernels' arithmetic under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): tests/sanitize_driver.c runs RHS evaluations,
steps, decision dumps and the boundary index maps over every boundary condition, side
tables with moving splits, 1D/2D/3D grids down to six points per line, gravity, the
scalar laws and an error path.  Any out-of-bounds access, leak or undefined
arithmetic aborts the run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "tests", "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def test_oracle_and_host_arithmetic_are_clean_under_sanitizers():
    gcc, gxx = shutil.which("gcc"), shutil.which("g++")
    if gcc is None or gxx is None:
        pytest.skip("gcc/g++ not available")
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "oracle"), "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1504_00731_amd", "csrc")]
    objs = []
    for src, cc, std in ((os.path.join(ROOT, "oracle", "wto_oracle.c"), gcc, "-std=c99"),
                         (os.path.join(ROOT, "tests", "sanitize_driver.c"), gcc, "-std=c99"),
                         (os.path.join(ROOT, "paper_1504_00731_amd", "csrc", "host_check.cpp"), gxx,
                          "-std=c++17")):
        obj = os.path.join(BUILD, "san_" + os.path.basename(src) + ".o")
        subprocess.run([cc, std, "-ffp-contract=off", "-fopenmp", "-Wno-unknown-pragmas", *SAN,
                        *inc, "-c", "-o", obj, src], check=True)
        objs.append(obj)
    exe = os.path.join(BUILD, "sanitize_driver")
    subprocess.run([gxx, "-fopenmp", *SAN, "-o", exe, *objs, "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "sanitized runs ok" in r.stdout
