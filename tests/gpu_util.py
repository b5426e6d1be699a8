"""Helpers shared by the GPU tests (test infrastructure)."""
import sys

import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(A):
    import paper_1408_5535_amd as P
    return P.DeviceCSR.from_scipy(A)


def as_np(t):
    return t.detach().cpu().numpy()
