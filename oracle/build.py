"""Build the oracle's shared library with the host C compiler.

Test infrastructure: compiles ``cggi_oracle.c`` (plain C, no GPU code) into
``libcggi_oracle.so`` next to it.  With CGGI_ORACLE_SANITIZE=1 in the
environment the library is built with the host compiler's address and
undefined-behaviour sanitizers (run the Python tests with the sanitizer
runtime preloaded, e.g. LD_PRELOAD=$(gcc -print-file-name=libasan.so) and
ASAN_OPTIONS=detect_leaks=0, since the interpreter itself is not
instrumented).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cggi_oracle.c")
LIB = os.path.join(HERE, "libcggi_oracle.so")


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    tmp = LIB + ".tmp"
    cmd = [cc, "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-strict-aliasing", "-o", tmp, SRC]
    if os.environ.get("CGGI_ORACLE_SANITIZE") == "1":
        cmd[1:2] = ["-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
