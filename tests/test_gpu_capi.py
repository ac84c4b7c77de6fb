"""The C ABI driven from a plain C program (tests/capi/solve_c.c, built with
the library): project, FBP, solve, history, data term and an argument error,
with no Python in between."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "capi", "solve_c")


def test_c_program_solves_through_the_abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/capi/solve_c is built with the library (paper_1009_1351_amd.build)"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert "capi ok" in r.stdout
