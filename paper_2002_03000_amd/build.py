"""Build libpperm.so (gfx950) in-tree with hipcc.

Flags that matter for results:
  -ffp-contract=off   no fused multiply-add: every IEEE operation of a decision
                      is rounded once, in the order written;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("pperm_kernels.hip", "pperm_api.hip", "pperm_server.hip",
                                                         "pperm_probe.hip")]
HEADERS = [os.path.join(HERE, "csrc", "pperm_internal.h"), os.path.join(ROOT, "include", "pperm.h"),
           os.path.join(ROOT, "include", "pperm_probe.h")]
LIB = os.path.join(HERE, "libpperm.so")
ARCH = os.environ.get("PPERM_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 2) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
               "-ffp-contract=off", "-fno-fast-math",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
