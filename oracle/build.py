"""Compile the CPU oracle (oracle.c) into liboracle.so with gcc.

Test infrastructure: the product library never builds against or links this.
Flags: -O2 with -ffp-contract=off so that every multiply and add of the
oracle rounds on its own, in the order the source writes it; OpenMP for the
plane loops (the loop bodies do not depend on the thread count).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, sanitize=False):
    """sanitize=True builds with AddressSanitizer and UndefinedBehaviorSanitizer
    (load it with gcc's libasan preloaded, ASAN_OPTIONS=detect_leaks=0)."""
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"] + san + \
          ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
