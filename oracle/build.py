"""Build the CPU oracle shared library (test infrastructure only).

The oracle is compiled with contraction and fast-math disabled so that every
operation is the IEEE double operation written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pn_oracle.cpp")
LIB = os.path.join(HERE, "libpn_oracle.so")

CMD = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c++17", "-Wall", "-Wextra",
       "-shared", "-fPIC", "-pthread", SRC, "-o", LIB]


# Host sanitizers for a checking build (plain g++, CPU code only).
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str = None, sanitize: bool = False) -> str:
    """Compile pn_oracle.cpp into libpn_oracle.so next to it (or into `out`);
    return the path.  sanitize=True adds AddressSanitizer and
    UndefinedBehaviorSanitizer instrumentation."""
    dst = out or LIB
    tmp = dst + ".tmp"
    cmd = CMD[:-2] + (SANITIZE if sanitize else []) + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, dst)
    return dst


def ensure_built() -> str:
    """Build only when the library is missing or older than its source."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        return build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
