"""Compile the synthetic-collection generator (plain C, host only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libssjgen.so")


# Host sanitizers for a checking build (gcc only, no GPU code here).
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
            "-g"]


def build(verbose: bool = False, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the library to ``out`` (default: next to the source); with
    ``sanitize``, with AddressSanitizer and UndefinedBehaviorSanitizer."""
    src = os.path.join(HERE, "ssjgen.c")
    lib = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-Wno-unused-parameter", *(SANITIZE if sanitize else []), src, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
