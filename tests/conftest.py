import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests that run the full-size workloads go last so a failure there hides nothing, and
    # the static-scratch entry point's file after them.
    items.sort(key=lambda it: (2 if "test_zz_" in it.nodeid else 1 if "full" in it.name else 0))
