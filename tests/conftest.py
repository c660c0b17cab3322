import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def oracle():
    import oracle as orc
    orc.build()
    return orc


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype):
    """numpy -> device tensor of `dtype` (torch.float32 / torch.float64)."""
    import torch
    return torch.from_numpy(np_contig(x)).to(device="cuda", dtype=dtype)


def np_contig(x):
    import numpy as np
    return np.ascontiguousarray(x)


def to_np(t):
    import numpy as np
    return t.detach().to("cpu", dtype=__import__("torch").float64).numpy().astype(np.float64)


def rounded(x, dtype):
    """The values a device tensor of `dtype` holds for x, back in float64."""
    import numpy as np
    import torch
    return x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x.astype(np.float64)
