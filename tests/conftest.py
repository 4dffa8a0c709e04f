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


_ONEPATCH = {}


def oracle_onepatch(problem, eps, tol_id=1e-12):
    """(Tables, OnePatch) of the oracle's full precompute, computed once per
    session for each (problem, eps, tol_id)."""
    from oracle import tables
    key = (problem, eps, tol_id)
    if key not in _ONEPATCH:
        tab, op, _ = tables.compute(problem, eps, 15, tol_id)
        _ONEPATCH[key] = (tab, op)
    return _ONEPATCH[key]
