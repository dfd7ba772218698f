"""Build the gfx950 library ``libflt.so`` (and, for tests, the CPU build of
the same kernel bodies, ``libflt_emu.so``) in-tree.

    python -m paper_1606_03255_amd.build            # library
    python -m paper_1606_03255_amd.build --emu      # library + CPU test build
    python -m paper_1606_03255_amd.build --emu-asan # library + CPU test build under ASan/UBSan
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libflt.so")
EMU = os.path.join(HERE, "libflt_emu.so")
EMU_ASAN = os.path.join(HERE, "libflt_emu_asan.so")
ARCH = os.environ.get("FLT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INC, "-I" + CSRC,
]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_lib(jobs=3):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = ["kernels.hip", "laplace.hip", "xi.hip", "api.cpp", "plan_host.cpp", "laplace_plan.cpp", "xi_plan.cpp"]
    objs = []
    procs = []
    for s in srcs:
        o = os.path.join(objdir, s + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = ["hipcc"] + HIP_FLAGS + lang + ["-c", os.path.join(CSRC, s), "-o", o]
        print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(o)
    rcs = [p.wait() for p in procs]
    if any(rcs):
        raise RuntimeError("compilation failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def build_emu(sanitize=False):
    """The CPU build of the kernel bodies (host compiler only).  sanitize=True
    builds it with AddressSanitizer and UndefinedBehaviorSanitizer into
    libflt_emu_asan.so; a process loading it needs libasan preloaded (see
    tests/test_cpu_build.py)."""
    out = EMU_ASAN if sanitize else EMU
    tmp = out + ".tmp%d" % os.getpid()
    extra = (["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-O1", "-DFLT_EMU_OMP_TEAMS"] if sanitize
             else ["-O2"])
    _run(["g++", "-g", "-std=c++17", "-fopenmp", "-fPIC", "-shared"] + extra + ["-I" + INC, "-I" + CSRC,
          os.path.join(CSRC, "emu.cpp"), os.path.join(CSRC, "plan_host.cpp"), os.path.join(CSRC, "laplace_plan.cpp"),
          os.path.join(CSRC, "xi_plan.cpp"), "-o", tmp])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build_lib()
    if "--emu" in sys.argv:
        build_emu()
    if "--emu-asan" in sys.argv:
        build_emu(sanitize=True)
