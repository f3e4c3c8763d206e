"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/hostcheck/build.py compiles the library's host code (the plan runtime, the
server, the filter catalogue and the host side of every kernel launch wrapper) for the
host with both sanitizers and links it against a model of the HIP stream, event and
graph-capture calls (tests/hostcheck/hip_model.cpp). The driver
(tests/hostcheck/driver.cpp) runs every C ABI call sequence on chains, stars, bushy and
binary trees of up to sixteen relations, 3- and 4-cycles, 4-cliques and a refused cyclic shape, in
recorded-graph, eager and profiling modes, with the asynchronous calls, filter inserts,
the filter catalogue (a plan destroyed after its context included) and a three-slot
server. It fails on any sanitizer report, any call that fails unexpectedly, and any
breach of the capture rules the model checks (an unjoined fork, a wait across captures
or on an event recorded outside the capture, a synchronisation inside a capture, use of
a destroyed stream or event, a kernel grid or block out of range).
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "hostcheck"))

pytestmark = pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/bin/clang++"), reason="needs the ROCm clang")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    import build
    return build.build(str(tmp_path_factory.mktemp("hostcheck")))


@pytest.mark.parametrize("scenario", ["chain", "star", "bushy", "binary", "chain12", "sixteen", "cycles",
                                      "updates", "fcache", "server", "errors", "static",
                                      "batch", "maintain"])
def test_scenario_clean_under_sanitizers(checker, scenario):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([checker, scenario], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert "scenario %-8s failures 0 violations 0" % scenario in out, out[-3000:]


def test_model_flags_an_unjoined_fork(tmp_path):
    """The capture model itself: a fork left unjoined at the end of a capture, and a wait
    on an event recorded outside the capture, are reported."""
    src = tmp_path / "probe.cpp"
    src.write_text(r'''
#include <hip/hip_runtime.h>
#include <cstdio>
extern "C" int hipmodel_violations();
__global__ void k() {}
int main() {
    hipStream_t a, b; hipEvent_t e, x;
    hipStreamCreateWithFlags(&a, hipStreamNonBlocking); hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
    hipEventCreateWithFlags(&e, hipEventDisableTiming); hipEventCreateWithFlags(&x, hipEventDisableTiming);
    hipEventRecord(x, a);
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipEventRecord(e, a);
    hipStreamWaitEvent(b, e, 0);
    hipLaunchKernelGGL(k, dim3(1), dim3(64), 0, b);
    hipStreamWaitEvent(a, x, 0);
    hipGraph_t g; hipError_t r = hipStreamEndCapture(a, &g);
    std::printf("end %d violations %d\n", (int)r, hipmodel_violations());
    return 0;
}
''')
    import build
    objs = []
    for s, lang in [(str(src), ["-x", "hip", "--cuda-host-only", "--offload-arch=gfx950"]),
                    (os.path.join(HERE, "hostcheck", "hip_model.cpp"),
                     ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"])]:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        subprocess.run([build.CLANG, *lang, "-O0", "-std=c++17", "-c", s, "-o", o], check=True)
        objs.append(o)
    fat = tmp_path / "fat.c"
    names = [l.split()[-1] for l in subprocess.run(["nm", "-u", objs[0]], capture_output=True, text=True,
                                                    check=True).stdout.splitlines()
             if l.split() and l.split()[-1].startswith("__hip_fatbin")]
    fat.write_text("".join("const char %s[16] = {0};\n" % n for n in names))
    exe = str(tmp_path / "probe")
    subprocess.run([build.CLANG, "-pthread", "-o", exe, *objs, "-x", "c", str(fat)], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert "waits on an event recorded outside the capture" in out.stderr
    assert "unjoined capture" in out.stderr
    assert "end 904 violations 2" in out.stdout, out.stdout + out.stderr


def test_batch_capture_clean_when_enabled(tmp_path):
    """The batch recording path (switched off in the library build) compiled in with
    SJ_BATCH_ENABLED=1 and run under the sanitizers and the capture model: every fork
    joined, no isolation breach, no memory error."""
    import build
    exe = build.build(str(tmp_path / "hc_batch"), defines=("SJ_BATCH_ENABLED=1",))
    r = subprocess.run([exe, "batch"], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1"))
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "scenario batch    failures 0 violations 0" in out
