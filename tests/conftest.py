import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O

    O.build()
    return O


def pytest_sessionfinish(session, exitstatus):
    """Write the worst error/bound ratio of every parity comparison that ran."""
    import json

    try:
        from _util import MARGINS
    except ImportError:
        return
    out = os.environ.get("KUBO_MARGINS_DIR")
    if not MARGINS or not out:
        return
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "parity_margins.json"), "w") as f:
        json.dump(MARGINS, f, indent=1)
