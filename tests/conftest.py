import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _build_missing():
    """Build whatever native library is missing (never rebuilds a present
    one: the GPU tests use the libraries as built, wherever they run)."""
    import oracle
    from paper_1401_6235_amd import build as hipbuild
    from paper_1401_6235_amd import workloads
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    if not os.path.exists(workloads.LIB_PATH):
        workloads.build()
    if not os.path.exists(hipbuild.LIB_PATH):
        hipbuild.build()


_build_missing()


def pytest_collection_modifyitems(config, items):
    """Skip GPU tests at once (before any input is generated) when no GPU is
    visible."""
    import pytest
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover - torch missing
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
