import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run, opt-in with LBM_SLOW_PINS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LBM_SLOW_PINS") == "1":
        return
    skip = pytest.mark.skip(reason="long oracle run; set LBM_SLOW_PINS=1 to run it")
    for it in items:
        if "slow" in it.keywords and "gpu" not in it.keywords:
            it.add_marker(skip)
