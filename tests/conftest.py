import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_sessionstart(session):
    # one per-eps table cache for the whole session (the library reads NCE_CACHE)
    import tempfile
    os.environ.setdefault("NCE_CACHE", tempfile.mkdtemp(prefix="nce_cache_"))
