import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # The CPU-side helper libraries are built only when absent; the build step
    # (__graft_entry__.build) always rebuilds them.
    import datagen
    import oracle
    for mod in (datagen, oracle):
        if not os.path.exists(mod._SO):
            mod.build()


@pytest.fixture(scope="session")
def gpu():
    """The GPU library bound to cuda:0; fails loudly if the HIP build is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a gpu-marked test ran without a visible GPU")
    import paper_2502_09541_amd as vx
    return vx
