"""Helpers shared by the GPU tests (marshalling and comparisons only)."""
import contextlib
import os
import sys

import numpy as np
import torch

from paper_2211_15716_amd import igg

PER = (1, 1, 1)


def say(*a):
    """Name the case on stdout before a GPU step, flushed."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@contextlib.contextmanager
def grid(n, periods=PER, overlaps=(2, 2, 2), zmarch_min=0, dims=(1, 1, 1)):
    """The global grid for one test.  zmarch_min is the smallest region the
    z-march kernels take (read at init): 0 sends every region through them,
    as the large grids do, so small test grids exercise their tiling; None
    keeps the library's default (small regions on the box kernels)."""
    nx, ny, nz = n
    key = "IGG_ZMARCH_MIN_POINTS"
    old = os.environ.get(key)
    if zmarch_min is None:
        os.environ.pop(key, None)
    else:
        os.environ[key] = str(zmarch_min)
    try:
        igg.init_global_grid(nx, ny, nz, dims=dims, periods=periods, overlaps=overlaps)
    finally:
        if old is None:
            os.environ.pop(key, None)
        else:
            os.environ[key] = old
    try:
        yield
    finally:
        torch.cuda.synchronize()
        igg.finalize_global_grid()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy()


def inner(a):
    return a[1:-1, 1:-1, 1:-1]


def rel_max_err(a, b):
    a, b = inner(np.asarray(a, np.float64)), inner(np.asarray(b, np.float64))
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
