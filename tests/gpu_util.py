"""Helpers for the GPU tests: device guard, progress marks, tensor <-> numpy."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

PROGRESS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "gpurun_out", "gpu_progress.log")


def announce(msg: str) -> None:
    """Name the case about to touch the GPU, on stderr (uncaptured) and in a
    progress file, flushed before the GPU step runs."""
    line = "[gpu-case] %s\n" % msg
    sys.__stderr__.write(line)
    sys.__stderr__.flush()
    try:
        os.makedirs(os.path.dirname(PROGRESS), exist_ok=True)
        with open(PROGRESS, "a") as f:
            f.write(line)
    except OSError:
        pass


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_0811_2535_amd as lf
    lf.lib()  # raises LibraryNotBuilt: never fall back
    return torch


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy()
