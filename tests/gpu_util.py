"""Helpers shared by the GPU tests: device transfer, comparisons, progress."""
import sys
import time

import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").contiguous()


def host(t):
    return t.detach().to("cpu").double().numpy()


def rel_max(a, b):
    """max |a - b| / max |b|."""
    d = np.abs(np.asarray(a) - np.asarray(b)).max()
    s = np.abs(np.asarray(b)).max()
    return d / s if s > 0 else d


def say(*args):
    print("[%s]" % time.strftime("%H:%M:%S"), *args, flush=True)
    sys.stdout.flush()
