import os
import sys

import pytest


def _keep_freed_memory() -> None:
    # The oracle allocates volume-sized temporaries many times per step; serving them
    # from a heap that keeps freed memory avoids fresh page faults on every one. This
    # changes where host memory comes from, never a value.
    import ctypes

    try:
        libc = ctypes.CDLL("libc.so.6")
        libc.mallopt(-4, 0)              # M_MMAP_MAX
        libc.mallopt(-1, 2 ** 31 - 1)    # M_TRIM_THRESHOLD
    except OSError:
        pass


_keep_freed_memory()

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly when it cannot run."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2311_13177_amd import binding

    return binding.lib()
