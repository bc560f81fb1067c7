import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle comparison")


@pytest.fixture(scope="session")
def gpu():
    """The loaded HIP library; GPU tests fail loudly when it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_2505_22797_amd import mpik
    return mpik


@pytest.fixture(autouse=True)
def bounds_checks_clean(request):
    """With the bounds-checked build loaded (MPIK_LIBRARY=libmpik_check.so),
    every plan a GPU test closes must report a zero check word."""
    yield
    if "gpu" not in request.keywords:
        return
    mpik = sys.modules.get("paper_2505_22797_amd.mpik")
    if mpik is None:
        return
    import gc
    gc.collect()
    failures = list(mpik.CHECK_FAILURES)
    mpik.CHECK_FAILURES.clear()
    assert not failures, f"bounds checks failed in the kernels: {failures}"
