"""Build the FP64 CPU oracle (``oracle.c`` -> ``liboracle.so``) with gcc.

Test infrastructure: the oracle is the checker of the HIP path, never part of
it.  Plain ``-O2`` without fast-math so that every operation is rounded as
written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


SAN_LIB = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build,
    liboracle_san.so (loaded instead of liboracle.so when ORACLE_LIB names
    it; the process must preload libasan)."""
    out = SAN_LIB if sanitize else LIB
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wextra"] + san + ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
