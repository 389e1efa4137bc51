"""The wavefront-per-block mapping (ballot per bit plane) computes the same
bit planes as the library's lane-per-block block code; the probe also times
both mappings (printed; the instruction counts come from a rocprofv3 run of
the same program)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "probe", "mapping_probe")


def test_wave_per_block_planes_equal_the_library_block_code():
    if not os.path.exists(EXE):
        pytest.fail("tests/probe/mapping_probe is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "check: 1024 blocks, 0 of 32768 plane words differ" in r.stdout
    assert "folds differing: 0" in r.stdout
