"""The bounded pull's index arithmetic on the host: the per-site maps give, for
every site and population, the index and ghost face of the direct position
formula (x faces, y faces, corners, periodic axes through bounded kernels, grids
of one to nine cells per axis).  Built with hipcc for the host, no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_pull_maps_reproduce_the_direct_pull_index(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "pull_index_check")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_05280_amd", "csrc"), "-o", exe,
                           os.path.join(HERE, "pull_index_check.hip")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 mismatches" in r.stdout
