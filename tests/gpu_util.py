"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import os
import sys

import numpy as np
import pytest


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def G():
    """The HIP binding; where a GPU is present a missing library is an error, not a skip."""
    from paper_2511_22094_amd import lib
    return lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
