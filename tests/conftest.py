import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@pytest.fixture(scope="session", autouse=True)
def _private_tune_cache(tmp_path_factory):
    """Tuned plans made by the tests write their layout cache to a scratch
    file of the session, never to the user's cache directory."""
    old = os.environ.get("VG_TUNE_CACHE")
    os.environ["VG_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "tune.json")
    yield
    if old is None:
        os.environ.pop("VG_TUNE_CACHE", None)
    else:
        os.environ["VG_TUNE_CACHE"] = old


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests run only where a GPU is visible; elsewhere they are skipped, so
    # `-m "not gpu"` and a bare `pytest` behave on a CPU-only host.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
