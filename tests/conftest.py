import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    # The C generator and the oracle are plain gcc builds; build them here only
    # if they are missing (the GPU library is never built by the tests).
    import oracle
    import synth
    for mod in (synth, oracle):
        if not os.path.exists(mod._LIB_PATH):
            mod.build()
