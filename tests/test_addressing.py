"""The population addressing of the collide-stream row form, checked on the
CPU (tests/addressing_check.hip, built with hipcc for the host): its 32-bit
group-row offsets equal the 64-bit reference offsets and stay inside a
population buffer, on the benchmark lattices (every row) and on the largest
lattices the library accepts with the row form (2^31 nodes in rows of 256;
padded row count times 19 just below 2^32), and the row form is switched off
exactly where those offsets could overflow."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1004_2416_amd", "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("addr") / "addressing_check")
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, "-I", INCLUDE,
                    os.path.join(HERE, "addressing_check.hip"), "-o", out], check=True,
                   capture_output=True)
    return out


def run(checker, *shapes):
    args = [str(v) for s in shapes for v in s]
    r = subprocess.run([checker] + args, capture_output=True, text=True)
    print(r.stdout)
    return r


def test_benchmark_lattices_every_row(checker):
    r = run(checker, (128, 128, 128), (256, 128, 128), (64, 64, 64), (32, 32, 32), (27, 19, 18),
            (30, 20, 16), (1, 1, 2), (253, 4, 3))
    assert r.returncode == 0
    assert r.stdout.count(": ok") == 8


def test_largest_lattices_with_the_row_form(checker):
    # 2^31 nodes in rows of 256 (the most nodes ibm_lattice_bytes accepts);
    # rows of 4 with the padded row count times 19 just below 2^32
    r = run(checker, (256, 65536, 128), (4, 65535, 3449), (100, 21474, 1000))
    assert r.returncode == 0
    assert r.stdout.count(": ok") == 3


def test_row_form_off_where_offsets_could_overflow(checker):
    # rows of 4: 65535 x 3450 rows times 19 exceeds 2^32; rows of 300 do not
    # fit a wavefront
    r = run(checker, (4, 65535, 3450), (300, 64, 64))
    assert r.returncode == 0
    assert r.stdout.count("row form no") == 2
