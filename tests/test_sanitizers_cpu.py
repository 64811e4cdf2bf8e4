"""The library's host code under sanitizers, on the CPU: the index, DC3,
index-file, suffix-tree and request-loop tests run against a host-only
build instrumented with AddressSanitizer + UndefinedBehaviorSanitizer, and
the request-loop tests (several threads: submitters, the loop, the scatter
thread) against one instrumented with ThreadSanitizer.  Each run is a child
Python process with the sanitizer runtime preloaded; any report fails it.
A planted heap overflow and a planted data race, built the same way, check
first that each runtime reports what it should."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1303_3692_amd import build as B  # noqa: E402

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="needs hipcc")

ENV = {
    "address": {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1"},
    "thread": {"TSAN_OPTIONS": "halt_on_error=1:report_signal_unsafe=0"},
}
TESTS = {
    "address": ["tests/test_host.py", "tests/test_suffix_tree_cpu.py", "tests/test_server_cpu.py"],
    "thread": ["tests/test_server_cpu.py"],
}
PLANTED = {
    "address": ("""
        #include <cstdlib>
        extern "C" int planted(int i) { int *p = (int *)std::malloc(4 * sizeof(int)); p[i] = 1; int v = p[i]; std::free(p); return v; }
    """, "planted(4)", "heap-buffer-overflow"),
    "thread": ("""
        #include <thread>
        static int shared_counter = 0;
        extern "C" int planted(int k) {
            std::thread a([k] { for (int j = 0; j < k; j++) shared_counter++; });
            std::thread b([k] { for (int j = 0; j < k; j++) shared_counter++; });
            a.join(); b.join(); return shared_counter;
        }
    """, "planted(100000)", "data race"),
}


def child_env(kind, lib=None):
    env = dict(os.environ)
    env.update(ENV[kind])
    env["LD_PRELOAD"] = B.runtime_path(kind)
    if lib:
        env["SAMATCH_LIB"] = lib
    return env


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_sanitizer_reports_planted_bug(kind, tmp_path):
    src, call, report = PLANTED[kind]
    cpp = tmp_path / "planted.cpp"
    cpp.write_text(textwrap.dedent(src))
    so = tmp_path / "libplanted.so"
    flags = []
    for f in B.SANITIZERS[kind]:
        flags += ["-Xarch_host", f]
    subprocess.run([B.hipcc(), "-O1", "-g", "-fPIC", "-shared", *flags, str(cpp), "-o", str(so), "-lpthread"],
                   check=True)
    r = subprocess.run([sys.executable, "-c", f"import ctypes; ctypes.CDLL({str(so)!r}).{call}"],
                       env=child_env(kind), capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and report in r.stderr, r.stderr[-2000:]


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_code_under_sanitizer(kind):
    lib = B.build_sanitized(kind)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *TESTS[kind]], cwd=ROOT, env=child_env(kind, lib), capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr, tail
    assert " passed" in r.stdout, tail
