"""Host checks of the engine's layout code, built as small host programs
against the in-tree library: every problem's carve takes exactly the bytes
its dry run reports (the dry run sizes every workspace, batch block and
server allocation), so no carve writes past the block it was given; and the
fused tiling follows its documented rules."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1306_0645_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run_host(tmp_path, name):
    if not os.path.exists(os.path.join(LIBDIR, "libfld.so")):
        pytest.skip("libfld.so not built")
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / name)
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(LIBDIR, "csrc"),
                    os.path.join(ROOT, "tests", "host", name + ".cpp"), "-o", exe,
                    "-L", LIBDIR, "-lfld", "-Wl,-rpath," + LIBDIR],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert re.search(r"(^|\s)0 mismatches", r.stdout), r.stdout


def test_dry_run_carve_equals_carve(tmp_path):
    _run_host(tmp_path, "carve_sizes")


def test_fused_tiling_rules(tmp_path):
    _run_host(tmp_path, "tile_rules")
