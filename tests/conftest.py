import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")



@pytest.fixture(autouse=True)
def _seed_global_rngs():
    """Every test starts from the same global random state, whichever tests
    ran before it in the process (the inputs of a test do not depend on the
    order or the subset that is run)."""
    import numpy as np
    import torch
    torch.manual_seed(1234)
    np.random.seed(1234)
    yield
