import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def parity_report():
    """Records per-result error figures (max amplitude error, 1 - fidelity)
    into the JSON-lines file named by OWQS_PARITY_REPORT, when set."""
    import json

    path = os.environ.get("OWQS_PARITY_REPORT")

    def record(name, **fields):
        if path:
            with open(path, "a") as fh:
                fh.write(json.dumps({"case": name, **fields}) + "\n")

    return record
