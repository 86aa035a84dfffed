import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _gpu_available():
    # counts devices without initialising the GPU runtime in this process
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        # the full-size tracking frames are rendered by a pool of forked
        # workers; forking a process whose GPU runtime is initialised is not
        # safe, so they are rendered here, before any test touches the GPU
        # (the sequence object is cached and the tests reuse it)
        if any(item.fspath.basename == "test_gpu_fullsize.py" for item in items):
            import synth
            seq = synth.c2_sequence(n_frames=100, map_size=1_000_000)
            seq.prefetch(range(50), workers=max(1, min(16, len(os.sched_getaffinity(0)))))
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
