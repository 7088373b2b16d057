"""Builds the sequential C++ driver of the triangulation code (tests/mesh_driver.cpp with
csrc/mesh_star.hpp, predicates.hpp and the host triangulation delaunay.cpp) for the CPU
tests, optionally with AddressSanitizer and UndefinedBehaviorSanitizer. Helpers only: no
test lives here."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_00758_amd", "csrc")

SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]


def build_driver(out_dir, sanitize=False):
    """Path of the built driver; None when g++ is not available."""
    if shutil.which("g++") is None:
        return None
    out = os.path.join(str(out_dir), "mesh_driver" + ("_san" if sanitize else ""))
    flags = SANITIZE if sanitize else ["-O2"]
    cmd = (["g++", "-std=c++17", "-Wall", "-Wextra"] + flags +
           [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
            os.path.join(ROOT, "tests", "mesh_driver.cpp"), os.path.join(CSRC, "delaunay.cpp"), "-o", out])
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def run_driver(driver, text, env=None):
    """Runs the driver on ``text`` (stdin); returns stdout. Fails on a non-zero exit."""
    res = subprocess.run([driver], input=text, capture_output=True, text=True, env=env)
    if res.returncode != 0:
        raise AssertionError(f"driver exited with {res.returncode}:\n{res.stderr[-4000:]}")
    return res.stdout
