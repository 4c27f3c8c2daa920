"""Band plan of the population scratch (host logic, no GPU): the plan
builder of the library, compiled with g++ beside a checker, must gather every
destination row once, after the reconstruction of every band within reach and
before that band's slot is filled again, and keep the scratch within the
budget until bands of one tile row do not fit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_band_plans(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2508_06911_amd", "csrc"),
                    "-o", exe, os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(ROOT, "paper_2508_06911_amd", "csrc", "lelbm_plan.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and "ALL OK" in r.stdout
