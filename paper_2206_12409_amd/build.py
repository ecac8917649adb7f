"""Build the gfx950 shared library libvsie.so in-tree with hipcc.

    python -m paper_2206_12409_amd.build        (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvsie.so")
BUILD = os.path.join(HERE, "_build")

HIP_SOURCES = ["kernels.hip", "vsie_api.hip", "dense_lu.hip", "cnn.hip", "learned.hip"]
HOST_SOURCES = ["setup_host.cpp", "setup_compress.cpp"]
ARCH = os.environ.get("VSIE_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=4):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-I" + CSRC]
    # packed FP32 instructions stay disabled for every HIP translation unit
    device = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    cmds, objs = [], []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([hipcc] + common + device + ["-ffp-contract=fast", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([hipcc] + common + ["-ffp-contract=off", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    procs = []
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        procs.append(subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        while len([p for p in procs if p.poll() is None]) >= jobs:
            procs[0].wait()
    errors = []
    for c, p in zip(cmds, procs):
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            errors.append(" ".join(c) + "\n" + out)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
