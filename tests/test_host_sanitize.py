"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(tests/native/abi_driver.cpp, built by paper_2307_12585_amd.build with the
sanitizers on the host pass only).  Without a GPU: the argument checks that
need no device (NULL contexts and arguments, a device index that does not
exist), with leak checking."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "abi_driver_san")
SUPP = os.path.join(ROOT, "tests", "native", "lsan_rocm.supp")


def sanitizer_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={SUPP}"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def run_driver(mode, timeout):
    if not os.path.exists(EXE):
        from paper_2307_12585_amd.build import build
        build()
    r = subprocess.run([EXE, mode], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=sanitizer_env(), timeout=timeout, cwd=os.path.dirname(EXE))
    return r.returncode, r.stdout


def assert_clean(rc, out):
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out
    assert "runtime error:" not in out, out
    assert "FAIL" not in out, out
    assert rc == 0 and "abi driver ok" in out, out


def test_abi_argument_checks_without_device_under_sanitizers():
    rc, out = run_driver("nodevice", 120)
    assert_clean(rc, out)
