"""Host check (CPU) of the row classification of boxes with walls or open
faces (plain rows and their x-end cells) that the sweep and reverse-step
kernels use: compiled from tests/native/plain_rows.cpp against the library's
internal header, and compared there with a brute-force reading of the pull
rule."""
import os
import subprocess
import tempfile

from paper_2310_14746_amd import build as hbuild

HERE = os.path.dirname(os.path.abspath(__file__))


def test_plain_rows_and_x_ends_match_the_pull_rule():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "plain_rows")
        subprocess.check_call([hbuild.hipcc(), "-O1", "-std=c++17", os.path.join(HERE, "native", "plain_rows.cpp"),
                               "-o", exe], stderr=subprocess.DEVNULL)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failed" in r.stdout
