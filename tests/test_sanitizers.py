"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer (host only; no GPU
code is built with them):

* the oracle (oracle/sem_oracle.c) built with -fsanitize=address,undefined and loaded,
  through SEM_ORACLE_LIB, by a child pytest running the oracle's pins
  (tests/test_oracle_pins.py) with the sanitizer runtimes preloaded;
* libsem's host setup (csrc/host_setup.cpp: GLL space, box mesh, gather-scatter and
  element-order maps, the Schwarz eigensolver, the thread pool) linked with
  tests/sanitize_host_setup.cpp, which drives it on regular and irregular inputs.

Both builds use -fno-sanitize-recover=all, so any finding ends the run with a non-zero
status."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.timeout(600)
def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", *SAN, "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-std=c11", "-D_GNU_SOURCE", "-o", lib, os.path.join(ROOT, "oracle", "sem_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", SEM_ORACLE_LIB=lib, PYTHONPATH=ROOT,
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=580)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]


@pytest.mark.timeout(300)
def test_host_setup_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_setup_san")
    csrc = os.path.join(ROOT, "paper_2107_01243_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", csrc, "-o", exe, os.path.join(HERE, "sanitize_host_setup.cpp"),
                    os.path.join(csrc, "host_setup.cpp"), "-lpthread"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=280,
                       env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ok" in r.stdout
