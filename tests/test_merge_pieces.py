"""Host check of the merge's indexing: for every voxel of a target block and
every (block size, reach) shape the kernels serve -- 2R > B included -- the
candidate list (merge_candidate) names exactly the neighbouring regions that
cover the voxel, and pbase / the compile-time piece bases give the voxel's
element in each region's piece-ordered partial sums, as counted out directly.
The check program (tests/merge_pieces_check.cpp) is built for the host with
hipcc from the library's own header; no GPU is used."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_merge_candidates_and_piece_offsets_match_direct_enumeration():
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "merge_pieces_check")
        r = subprocess.run([hipcc, "-O1", "-std=c++17",
                            "-I", os.path.join(ROOT, "paper_1909_04631_amd", "csrc"),
                            "-I", os.path.join(ROOT, "include"),
                            os.path.join(ROOT, "tests", "merge_pieces_check.cpp"), "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout
    assert "B=4 R=4" in out.stdout and "B=2 R=2" in out.stdout   # the 2R > B shapes
