"""Helpers for the GPU parity tests (oracle on the CPU, library on the GPU)."""
import os
import sys

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("a GPU test was selected but no GPU is visible")


def announce(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(got, want):
    got = got.detach().cpu().numpy() if isinstance(got, torch.Tensor) else got
    scale = np.max(np.abs(want))
    return float(np.max(np.abs(got - want)) / (scale if scale > 0 else 1.0))


class engine_path:
    """Force the four-step path for 1D plans created inside the block."""
    def __enter__(self):
        os.environ["AZRBF_ENGINE"] = "1"

    def __exit__(self, *a):
        os.environ.pop("AZRBF_ENGINE", None)
