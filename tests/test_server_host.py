"""The query server's host logic under AddressSanitizer, UndefinedBehavior-
Sanitizer and ThreadSanitizer, on the CPU.

dtn_server.cpp is compiled against a host-only stand-in of the HIP runtime
(tests/server_host/: streams are worker threads, stream capture records
closures into graphs, graph-owned allocations are poisoned between replays)
and stub launchers whose outputs are simple functions of their inputs, then
driven through a serving trace: queries of 1..512 boundary points arriving
about 200 us apart, several streams, direct launches and graph replay
(enabled for this build only), patch and point modes.  Every answer is
checked against the query's own points, every padding row read by a stub
"kernel" must be a valid descriptor, and the server is also destroyed with
queries queued and in flight.  Graph replay must never begin a capture on a
stream that has unfinished work, even when host functions take longer to
complete (FAKE_HOSTFN_TAIL_US)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "server_host")
SOURCES = [os.path.join(HOST, f) for f in ("fake_hip.cpp", "stubs.cpp", "drive.cpp")] + \
    [os.path.join(ROOT, "paper_1210_1491_amd", "csrc", "dtn_server.cpp")]
FLAGS = ["-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer", "-I" + HOST,
         "-I" + os.path.join(ROOT, "paper_1210_1491_amd", "csrc"), "-DDTN_SERVER_GRAPH_REPLAY=1"]
CLANG = "/opt/rocm/llvm/bin/clang++"
MODES = [(4, 0, 0), (4, 1, 0), (4, 0, 1), (4, 1, 1), (16, 1, 0), (1, 1, 0)]


def _build(tmp_path_factory, name, compiler, sanitize):
    out = str(tmp_path_factory.mktemp("server_host") / name)
    subprocess.run([compiler, *FLAGS, sanitize, *SOURCES, "-o", out], check=True, capture_output=True, timeout=300)
    return out


def _run(exe, mode, tail_us=0, queries=60, seed=7):
    env = dict(os.environ, FAKE_HOSTFN_TAIL_US=str(tail_us), ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *map(str, mode), str(queries), str(seed), "512"], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "failures 0" in r.stdout and "(0 on a stream with unfinished work)" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def asan_exe(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    return _build(tmp_path_factory, "drive_asan", "g++", "-fsanitize=address,undefined")


@pytest.fixture(scope="module")
def tsan_exe(tmp_path_factory):
    # gcc 11's ThreadSanitizer does not intercept pthread_cond_clockwait
    # (condition waits with a timeout on the steady clock) and reports the
    # waiting thread as still holding the mutex; the ROCm clang runtime does.
    if not os.path.exists(CLANG):
        pytest.skip("no clang with a ThreadSanitizer runtime")
    return _build(tmp_path_factory, "drive_tsan", CLANG, "-fsanitize=thread")


@pytest.mark.parametrize("mode", MODES)
def test_server_host_logic_under_asan_ubsan(asan_exe, mode):
    out = _run(asan_exe, mode, tail_us=500 if mode[1] else 0)
    if mode[1]:
        assert " 0 graph launches" not in out


@pytest.mark.parametrize("mode", MODES[:4])
def test_server_host_logic_under_tsan(tsan_exe, mode):
    _run(tsan_exe, mode, tail_us=300 if mode[1] else 0, queries=40)
