"""The C boundary used from a C program with no Python in it
(tests/c_abi/hg_c_example.cpp, built by the package's build step): setup,
channels, counts, an argument error and finish on one small field; constant
channels must come out constant and empty cells NaN.  Run as a child
process."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "hg_c_example")


def test_c_program_grids_through_the_abi():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "c abi ok" in r.stdout
