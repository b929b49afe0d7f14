"""The C ABI used from plain C, with no Python or torch in the process:
tests/c_abi/free_fall.c (built by __graft_entry__.build()) checks free fall
against its closed form and a tool-pressed run's status."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def test_plain_c_client():
    exe = os.path.join(HERE, "c_abi", "free_fall")
    assert os.path.exists(exe), "build() compiles tests/c_abi/free_fall.c"
    print("plain-C client: 8,000 particles, 64^3, 40 free-fall + 40 pressed substeps", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")
