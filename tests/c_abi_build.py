"""Build helper for tests/c/abi_demo.c: gcc against include/pf.h and the
in-tree libpfiso.so (no Python or torch in the program)."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2110_12448_amd")


def build_demo(out_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        return None, "gcc not found"
    cmd = [gcc, "-O2", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_demo.c"), "-L", PKG, "-lpfiso",
           "-Wl,-rpath," + PKG, "-L/opt/rocm/lib", "-Wl,-rpath-link,/opt/rocm/lib", "-lm",
           "-o", out_path]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, r.stderr
