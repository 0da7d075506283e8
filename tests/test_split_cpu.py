"""Host check (CPU) of the interior/shell decomposition of boxes with walls or
open faces that the adjoint sweep launches: compiled from
tests/native/split_coverage.cpp against the library's internal header."""
import os
import subprocess
import tempfile

from paper_2310_14746_amd import build as hbuild

HERE = os.path.dirname(os.path.abspath(__file__))


def test_split_covers_every_cell_once():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "split_coverage")
        subprocess.check_call([hbuild.hipcc(), "-O1", "-std=c++17", os.path.join(HERE, "native", "split_coverage.cpp"),
                               "-o", exe], stderr=subprocess.DEVNULL)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failed" in r.stdout
