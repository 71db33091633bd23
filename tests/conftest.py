import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def progress(msg: str) -> None:
    """Progress line for long GPU tests: straight to the terminal (past pytest's
    output capture), and appended to the file CBS_PROGRESS_LOG names, if set."""
    import sys
    import time
    line = f"[{time.strftime('%H:%M:%S')}] {msg}"
    try:
        sys.__stderr__.write(line + "\n")
        sys.__stderr__.flush()
    except Exception:
        pass
    path = os.environ.get("CBS_PROGRESS_LOG")
    if not path:
        return
    try:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "a") as f:
            f.write(line + "\n")
    except OSError:
        pass


@pytest.fixture(scope="session")
def report():
    return progress


@pytest.fixture(scope="session")
def orc():
    from oracle import core
    core.lib()
    return core
