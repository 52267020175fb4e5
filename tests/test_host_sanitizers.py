"""Host sanitizer run of the C code that has no GPU part: the CPU oracle
(oracle/wc_truss.c) and the input generators (graphgen/graphgen.c) are built with
AddressSanitizer and UndefinedBehaviorSanitizer into a temporary directory, and the
oracle's pins, the k-core oracle's pins and the generator tests run against those
builds in a child process (any sanitizer report aborts it)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _gcc_lib(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.slow
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    asan = _gcc_lib("libasan.so")
    ubsan = _gcc_lib("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    orc = str(tmp_path / "wc_truss_san.so")
    gen = str(tmp_path / "graphgen_san.so")
    subprocess.check_call(["gcc", *SAN, "-fPIC", "-shared", "-o", orc, os.path.join(ROOT, "oracle", "wc_truss.c")])
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-o", gen,
                           os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm"])
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": f"{asan}:{ubsan}",
        # the interpreter itself is not instrumented: its allocations are not leaks of ours
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "PKT_ORACLE_LIB": orc,
        "PKT_GRAPHGEN_LIB": gen,
        "OMP_NUM_THREADS": "2",
    })
    tests = ["tests/test_oracle_pins.py", "tests/test_kcore_oracle.py", "tests/test_graphgen.py",
             "tests/test_certificate.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout
    # the child really loaded the sanitized builds
    probe = subprocess.run([sys.executable, "-c",
                            "import oracle, graphgen; print(oracle._load()._name); print(graphgen._load()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert orc in probe.stdout and gen in probe.stdout
