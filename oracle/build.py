"""Build the plain-C FP64 oracle (test infrastructure) into oracle/libeb_oracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libeb_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "eb_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


CHECK = os.path.join(HERE, "_build", "sanitize_check")


def build_sanitize_check(verbose: bool = False) -> str:
    """The sanitizer driver (sanitize_check.c with the oracle, -fsanitize=address,undefined):
    built here so that a build compiles every C source of the oracle; tests/
    test_oracle_sanitized.py builds and runs its own copy."""
    os.makedirs(os.path.dirname(CHECK), exist_ok=True)
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", HERE, os.path.join(HERE, "eb_oracle.c"), os.path.join(HERE, "sanitize_check.c"),
           "-o", CHECK, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return CHECK


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_sanitize_check(verbose="-v" in sys.argv)
    print(LIB)
