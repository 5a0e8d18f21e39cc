"""Compile the CPU oracle (oracle.c) into oracle/liboracle.so with gcc.

Test infrastructure: the oracle is built with every product and sum rounded
on its own (no FMA contraction, no fast-math) so that it follows the
paper's C99 arithmetic.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


# A checking build of the same source with the address and
# undefined-behaviour sanitizers (host code only; built on request by the
# sanitizer test, which loads it into a child process with the ASan runtime
# preloaded).
SAN_LIB = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    flags = [f for f in CFLAGS if not (sanitize and f == "-O2")] + (SAN_FLAGS if sanitize else [])
    cmd = ["gcc", *flags, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
