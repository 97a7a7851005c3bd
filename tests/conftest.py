import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs (not part of the default suite)")


def pytest_collection_modifyitems(config, items):
    import pytest
    if os.environ.get("FGA_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="long oracle run; set FGA_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
