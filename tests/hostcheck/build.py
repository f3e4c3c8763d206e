"""Build the host-runtime checker: the library's host code (the runtime, the server,
the filter catalogue and the host side of the kernel launch wrappers) compiled for
the host only with AddressSanitizer and UndefinedBehaviorSanitizer, linked against the
HIP model (hip_model.cpp) and the scenario driver (driver.cpp).

    python tests/hostcheck/build.py [out_dir]     -> prints the executable's path
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2308_16370_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
CLANG = os.environ.get("HOSTCHECK_CXX", "/opt/rocm/llvm/bin/clang++")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
COMMON = ["-O1", "-g", "-std=c++17", "-pthread", "-I" + INCLUDE, "-I" + CSRC, *SAN]


def sources(csrc: str = CSRC):
    out = []
    for f in sorted(os.listdir(csrc)):
        if f.endswith(".hip"):
            out.append((os.path.join(csrc, f), ["-x", "hip", "--cuda-host-only", "--offload-arch=gfx950"]))
        elif f.endswith(".cpp"):
            out.append((os.path.join(csrc, f), ["-x", "hip", "--cuda-host-only", "--offload-arch=gfx950"]))
    out.append((os.path.join(HERE, "hip_model.cpp"), ["-x", "c++", "-D__HIP_PLATFORM_AMD__",
                                                      "-I/opt/rocm/include"]))
    out.append((os.path.join(HERE, "driver.cpp"), ["-x", "c++"]))
    return out


def build(out_dir: str, csrc: str = CSRC, defines=()) -> str:
    os.makedirs(out_dir, exist_ok=True)

    def one(item):
        src, lang = item
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        cmd = [CLANG, *lang, *COMMON, *["-D" + d for d in defines], "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(one, sources(csrc)))
    # the compiler names each translation unit's (here empty) device image by a hash;
    # define those symbols so the host-only objects link
    stub = os.path.join(out_dir, "fatbin_stubs.c")
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        for line in r.stdout.splitlines():
            parts = line.split()
            if parts and parts[-1].startswith("__hip_fatbin"):
                names.add(parts[-1])
    with open(stub, "w") as fh:
        for n in sorted(names):
            fh.write("const char %s[16] = {0};\n" % n)
    sobj = os.path.join(out_dir, "fatbin_stubs.o")
    subprocess.run([CLANG, "-x", "c", "-c", stub, "-o", sobj], check=True)
    exe = os.path.join(out_dir, "hostcheck")
    cmd = [CLANG, *SAN, "-pthread", "-o", exe, *objs, sobj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_build", "hostcheck")))
