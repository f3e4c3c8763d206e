"""Build libsievejoin.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsievejoin.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
SOURCES = ["sj_kernels.hip", "sj_join.hip", "sj_runtime.cpp", "sj_server.cpp", "sj_fcache.cpp", "sj_tri.hip",
           "sj_update.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, out: str = LIB, defines=(), csrc: str = CSRC) -> str:
    """Compile every source (in parallel) and link the shared library; returns its path.

    ``defines`` are extra ``-D`` tuning macros (the defaults are the tuned values);
    ``csrc`` is the source directory."""
    def snapshot():
        files = [os.path.join(csrc, f) for f in os.listdir(csrc)] + \
                [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
        return {f: os.stat(f).st_mtime_ns for f in files if os.path.isfile(f)}

    before = snapshot()
    with tempfile.TemporaryDirectory(prefix="sjbuild") as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip", "-pthread"] if src.endswith(".cpp") else []
            cmd = [HIPCC, *FLAGS, "-I" + INCLUDE, *["-D" + d for d in defines], *lang, "-c", os.path.join(csrc, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-4000:]))
            if verbose and r.stderr:
                print(r.stderr)
            return obj

        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        out_tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", out_tmp, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
        # a source edited while the objects compiled would leave objects built from
        # different versions of the shared headers in one library: refuse it
        if snapshot() != before:
            os.remove(out_tmp)
            raise RuntimeError("a source file changed during the build; build again")
        os.replace(out_tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
