import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle physics runs")


def _gpu_present() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_present():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(autouse=True)
def _single_pass_step_at_every_size(request, monkeypatch):
    """GPU tests run the single-pass D3Q27 step on their small grids too (LBM2P_FUSED=1), as the
    library takes it on large ones; by default small grids take the two-pass step. Tests of
    that size rule remove the variable themselves."""
    if "gpu" in request.keywords:
        monkeypatch.setenv("LBM2P_FUSED", "1")
    yield

