"""Build the gfx950 HIP library libpn_hip.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpn_hip.so")
SOURCES = [os.path.join(CSRC, "pn_kernels.hip"), os.path.join(CSRC, "pn_mlp.hip")]
HEADERS = [os.path.join(CSRC, "pn_device.h"), os.path.join(ROOT, "include", "pn.h")]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra=None) -> str:
    """Compile every HIP source into libpn_hip.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + (extra or []) + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def resource_usage() -> str:
    """Per-kernel VGPR/AGPR/SGPR/scratch/occupancy report from the compiler."""
    out = []
    for src in SOURCES:
        cmd = ["hipcc"] + FLAGS[:-4] + ["-c", "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage",
                                        "--cuda-device-only", "-I", os.path.join(ROOT, "include"), "-I", CSRC, src]
        cmd = [c for c in cmd if c not in ("-shared", "-fPIC")]
        out.append(subprocess.run(cmd, capture_output=True, text=True).stderr)
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--resources":
        print(resource_usage())
    else:
        print(build(verbose=True))
