import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The tests check the library's own shape choice (built-in table, defaults);
# an override left in the caller's environment would replace it.  Tests that
# exercise PWADV_TILE set it themselves.
os.environ.pop("PWADV_TILE", None)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


_REPORT = {}


@pytest.fixture(scope="session")
def report():
    """Session-wide dict of measured figures (errors against the oracle).
    Written as JSON to $PWADV_REPORT at the end of the session if set."""
    return _REPORT


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("PWADV_REPORT")
    if path and _REPORT:
        import json
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(_REPORT, fh, indent=1, sort_keys=True)


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Print the measured figures (per-form errors against the oracle) at the
    end of the run, so the run's own log carries them."""
    if not _REPORT:
        return
    import json
    terminalreporter.write_sep("-", "parity figures (errors against the FP64 oracle)")
    for key in sorted(_REPORT):
        terminalreporter.write_line("%s: %s" % (key, json.dumps(_REPORT[key], sort_keys=True, default=str)))
