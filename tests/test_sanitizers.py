"""The oracle (oracle/oracle.c) and the library's host setup code
(csrc/host_setup.cpp, through tests/host_driver.cpp) built with
AddressSanitizer and UndefinedBehaviorSanitizer, aborting on the first
report, running their CPU pins: the oracle's pins and the host-logic tests
in a child process that preloads the sanitizer runtime (Python itself is not
instrumented; leak checking is off)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    return subprocess.run(["gcc", "-print-file-name=" + name], stdout=subprocess.PIPE, text=True,
                          check=True).stdout.strip()


def test_oracle_and_host_setup_under_asan_ubsan():
    env = dict(os.environ)
    env.update({
        "ORACLE_SANITIZE": "1",
        "ESD_HOST_SANITIZE": "1",
        "LD_PRELOAD": _runtime("libasan.so") + " " + _runtime("libubsan.so"),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_host_logic.py")],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=900)
    tail = r.stdout[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error:" not in r.stdout, tail
    assert " passed" in tail
