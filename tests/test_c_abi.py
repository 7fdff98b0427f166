"""The C ABI from plain C: tests/c_abi_host.c is compiled with gcc against include/wqa.h,
linked with libwqa.so, and run on the host (host-only context); its output must agree
with the Python binding's view of the same space."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def wqa():
    import paper_1710_01048_amd as mod
    return mod


def test_plain_c_client(wqa, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    libdir = os.path.dirname(wqa.lib_path)
    exe = str(tmp_path / "c_abi_host")
    subprocess.run([gcc, "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_host.c"), "-o", exe, "-L", libdir, "-lwqa",
                    "-Wl,-rpath," + libdir], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.splitlines()
    sp = wqa.Space(3, 3, (4, 5, 6), device=None)
    assert out[0] == "rows %d slots %d points %d grid %d %d %d" % ((sp.n_rows, sp.slots_per_row, sp.points_per_row)
                                                                   + sp.grid_shape)
    x, w = sp.rules(wqa.MASS, 2)
    words = out[1].split()
    assert float(words[3]) == pytest.approx(w.sum(), rel=0, abs=1e-15) and float(words[6]) == x[0, 0]
    assert out[2].startswith("estate: wqa_assemble_mass")
    assert out[-1] == "ok"
