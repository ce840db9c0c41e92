import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Finish the GPU's queued work and release the library's live handles
    (contexts, trees, networks, photon maps, batches) while the HIP runtime
    is fully up, instead of leaving them to interpreter shutdown."""
    torch = sys.modules.get("torch")
    gpu = torch is not None and torch.cuda.is_initialized()
    if gpu:
        torch.cuda.synchronize()
    binding = sys.modules.get("paper_2107_11008_amd._sc")
    if binding is not None:
        binding._release_all()
    if gpu:
        torch.cuda.synchronize()
