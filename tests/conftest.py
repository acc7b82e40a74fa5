import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from tests import oracle_jobs  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "oracle_job(name): the test waits for a background oracle "
                                       "reference run (tests/oracle_jobs.py)")


def pytest_collection_finish(session):
    """Start the oracle jobs the selected tests need, so that they run while
    the other tests do."""
    if session.config.option.collectonly:
        return
    names = set()
    for item in session.items:
        for m in item.iter_markers("oracle_job"):
            names.update(m.args)
    oracle_jobs.start(sorted(names))


def pytest_sessionfinish(session, exitstatus):
    oracle_jobs.stop_all()
