import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture()
def rng():
    """A fresh generator per test, so results do not depend on test order."""
    import numpy as np
    return np.random.default_rng(2024)


import faulthandler  # noqa: E402

faulthandler.enable()
