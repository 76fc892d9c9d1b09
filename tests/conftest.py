import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libpolfed.so")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


def pytest_report_header(config):
    return f"polfed tests, root={ROOT}"


@pytest.fixture(autouse=True)
def _name_case(request):
    # name every test on stdout before it runs, so that a GPU run cut short
    # still shows which case was running
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[case] {request.node.nodeid}", flush=True)
    yield
