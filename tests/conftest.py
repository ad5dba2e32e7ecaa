import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (gfx950); runs through the C ABI of libmfs")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


def pytest_collection_modifyitems(config, items):
    # a gpu test without a visible device fails loudly instead of skipping.
    # slow tests (minutes of oracle CPU work, e.g. the 10^4-body sampled rows)
    # run only when MFS_SLOW=1 is set.
    if os.environ.get("MFS_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="minutes of oracle CPU work; run with MFS_SLOW=1")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
