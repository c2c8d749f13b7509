import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # CPU-side libraries are cheap to build; build them if a checkout lacks them.
    import oracle
    from paper_2505_02017_amd import scenes
    if not os.path.exists(oracle.lib_path()):
        oracle.build()
    if not os.path.exists(scenes.lib_path()):
        scenes.build()
