"""Build the host AddressSanitizer harness (tests/asan/harness.cpp) with the library's HIP
sources: AddressSanitizer on the host code only (-Xarch_host), the device code as in
libfpdlbm.so.  Output: tests/asan/_build/fpd_asan_harness."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2212_14153_amd import build as lib_build  # noqa: E402

OUT = os.path.join(HERE, "_build", "fpd_asan_harness")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    flags = [f for f in lib_build.FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [lib_build.hipcc(), *flags,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           f"-I{lib_build.INCLUDE}", f"-I{lib_build.CSRC}", "-o", OUT + ".tmp",
           *[os.path.join(lib_build.CSRC, s) for s in lib_build.SOURCES],
           os.path.join(HERE, "harness.cpp"), *lib_build.LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
