"""The C ABI used from a plain host program (examples/c_api.cpp): hipMalloc'd buffers,
no PyTorch.  The program checks its result against a dense sum it computes itself."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "examples", "c_api")


def test_example_source_uses_only_the_public_header():
    src = open(os.path.join(ROOT, "examples", "c_api.cpp")).read()
    includes = [l.split()[1] for l in src.splitlines() if l.startswith("#include")]
    assert '"spkadd.h"' in includes
    assert not any("csrc" in i or "internal" in i or "torch" in i for i in includes)


@pytest.mark.gpu
def test_c_api_example_runs():
    if not os.path.exists(EXAMPLE):
        pytest.fail("examples/c_api is not built (run __graft_entry__.build())")
    print("running", EXAMPLE, flush=True)
    res = subprocess.run([EXAMPLE], capture_output=True, text=True, timeout=90)
    assert res.returncode == 0, res.stderr
    assert res.stdout.startswith("ok "), res.stdout
    assert int(res.stdout.split()[1]) > 0
