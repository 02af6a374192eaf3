"""The library through its C ABI alone: a C program (tests/c/ace_c_demo.c)
compiled with gcc against include/ace.h and linked to libace.so, with no
Python or torch between it and the kernels.  Compiling it checks that the
header is plain C; running it on the GPU checks the results against the
oracle."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "ace_c_demo.c")
PKG = os.path.join(ROOT, "paper_2312_07010_amd")


def _compile(tmp_path):
    exe = str(tmp_path / "ace_c_demo")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           SRC, "-o", exe, "-L", PKG, "-lace", f"-Wl,-rpath,{PKG}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_header_is_plain_c_and_links(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libace.so")):
        pytest.skip("libace.so not built")
    assert os.path.exists(_compile(tmp_path))


@pytest.mark.gpu
def test_c_program_matches_oracle(tmp_path, orc):
    exe = _compile(tmp_path)
    n, eps, dt, steps = 40, 0.02, 1e-3, 25
    p = orc.Problem(2, [n, n], [0, 0], [1, 1], eps, dt, "HN")
    phi0 = np.random.default_rng(4).uniform(-0.9, 0.9, p.shape)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    phi0.tofile(fin)
    r = subprocess.run([exe, str(n), repr(eps), repr(dt), str(steps), str(fin), str(fout)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout)
    out = np.fromfile(fout)
    total = p.shape[0] * p.shape[1]
    phi, E, mx, mom = out[:total], out[total], out[total + 1], out[total + 2:]
    want, _, _ = p.run(phi0, steps)
    np.testing.assert_allclose(phi.reshape(p.shape), want, rtol=0, atol=1e-13)
    assert E == pytest.approx(p.energy(want), rel=1e-12)
    assert mx == pytest.approx(np.abs(want).max(), abs=1e-13)
    np.testing.assert_allclose(mom.reshape(p.shape), want, rtol=0, atol=1e-13)
