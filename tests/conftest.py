import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not (ROOT / "oracle" / "liborc.so").exists():
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding, on a machine with a GPU.  A missing library on a GPU
    machine is an error, not a skip."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2010_11540_amd import scpic
    scpic.load_library()
    torch.cuda.init()
    return scpic
