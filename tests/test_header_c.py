"""The public header as plain C: tests/header_c_check.c (C99, -Wall -Werror,
gcc) includes include/nadmm.h, links against the built libnadmm.so and calls
its host-only entry points (version, digest, status strings, workspace
sizes, launch shapes, argument errors) from C.  No device is touched."""
import os
import shutil
import subprocess

import pytest

from paper_2109_12688_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_compiles_and_links_as_c99(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2109_12688_amd.build import build
        build()
    lib_dir = os.path.dirname(os.path.abspath(_lib.LIB_PATH))
    exe = str(tmp_path / "header_c_check")
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "header_c_check.c"),
           "-L", lib_dir, "-l:" + os.path.basename(_lib.LIB_PATH), "-Wl,-rpath," + lib_dir, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout + run.stderr
