import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(params=["run", "wave"])
def mttkrp_form(request):
    """Runs a test with each form of the MTTKRP kernel forced (each lane group on its own
    run of nonzeros, or a whole wave on one run), then restores the automatic choice."""
    from paper_1902_03317_amd._lib import lib
    lib.pasta_set_mttkrp_form({"run": 1, "wave": 2}[request.param])
    yield request.param
    lib.pasta_set_mttkrp_form(0)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
