import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False,
                     help="run the long CPU oracle checks (minutes each)")


def pytest_collection_modifyitems(config, items):
    import pytest
    if config.getoption("--runslow"):
        return
    skip = pytest.mark.skip(reason="long oracle run: pass --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
