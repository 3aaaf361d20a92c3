import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # plans take their tile shape from the autotuner's cache; a fresh cache per
    # session keeps the shape each test runs independent of what a host's
    # ~/.cache holds (tests that tune point the library at their own file)
    import tempfile
    os.environ["TGW_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="tgw_tune_"), "tune.json")
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; on a CPU-only host they are skipped
    # unless explicitly selected, in which case they fail loudly.
    markexpr = config.getoption("-m") or ""
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu or "gpu" in markexpr and "not gpu" not in markexpr:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
