"""Build libswe_hip.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswe_hip.so")
SOURCES = [os.path.join(CSRC, "swe_api.hip")]
DEPS = SOURCES + [os.path.join(CSRC, "swe_step.hpp"), os.path.join(CSRC, "swe_nest.hpp"),
                  os.path.join(CSRC, "swe_lc.hpp"),
                  os.path.join(os.path.dirname(HERE), "include", "swe.h")]

# Packed FP32 instructions are disabled on purpose: every FP32 operation is
# issued as a plain VALU instruction.  Multiply-adds are fused only within a
# single source expression (-ffp-contract=on, never across statements), so
# every tile shape (template instantiation) rounds every cell identically and
# results do not depend on the tile shape.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function"]


def build(verbose=False, resource_report=None, out=None, defines=()):
    """Compile the library (to `out`, default in-tree); `defines` are extra
    -D settings such as SWE_WAVES_PER_SIMD_F32=2."""
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-D" + d for d in defines] + ["-o", out or LIB] + SOURCES
    if resource_report:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if resource_report:
        with open(resource_report, "w") as f:
            f.write(res.stderr)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        raise RuntimeError("hipcc failed building %s" % (out or LIB))
    if verbose:
        sys.stderr.write(res.stderr)
    return out or LIB


if __name__ == "__main__":
    build(verbose=True, resource_report=sys.argv[1] if len(sys.argv) > 1 else None)
    print(LIB)
