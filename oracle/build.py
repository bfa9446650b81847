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


def build(verbose: bool = False) -> str:
    """Compile pn_oracle.cpp into libpn_oracle.so next to it; return the path."""
    tmp = LIB + ".tmp"
    cmd = CMD[:-1] + [tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    """Build only when the library is missing or older than its source."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        return build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
