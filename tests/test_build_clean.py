"""build() from a clean checkout: a copy of the tracked sources without any
built library must compile libpmc.so and import the package."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_build_from_clean_checkout(tmp_path):
    if shutil.which("hipcc") is None or shutil.which("git") is None:
        pytest.skip("needs hipcc and git")
    files = subprocess.run(["git", "ls-files", "-z"], cwd=ROOT, capture_output=True, check=True).stdout
    names = [f for f in files.decode().split("\0") if f]
    if not names:
        pytest.skip("not a git checkout")
    dst = tmp_path / "repo"
    for f in names:
        src = os.path.join(ROOT, f)
        if not os.path.isfile(src):
            continue
        out = dst / f
        out.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy2(src, out)
    assert not (dst / "paper_2108_03076_amd" / "libpmc.so").exists()
    code = "import __graft_entry__ as g; g.build(); import paper_2108_03076_amd as P; print(P.LIB_PATH)"
    r = subprocess.run([sys.executable, "-c", code], cwd=dst, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    lib = dst / "paper_2108_03076_amd" / "libpmc.so"
    assert lib.exists() and r.stdout.strip().endswith("libpmc.so")
