"""Time-loop drivers over the C-ABI library: the Fig. 1 loop (step, halo
update, swap), its FP32/FP16 forms, and the reverse sweep with
time-loop checkpointing behind a torch.autograd.Function.

Everything numeric runs in the library's kernels; this module only orders
calls, swaps buffers and keeps snapshots (device tensors).
"""
import math

import torch

from . import igg

DTYPES = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def to_device(arr, dtype=torch.float64, device="cuda"):
    """Upload a float64 numpy array and round it once to `dtype` on the device
    (round to nearest even)."""
    t = torch.from_numpy(arr).to(device=device)
    return t.to(dtype).contiguous()


def prepare_fields(T0, Ci, dtype=torch.float64, device="cuda", stream=None):
    """Device copies of T0 and Ci in `dtype` with their halos updated."""
    T = to_device(T0, dtype, device)
    C = to_device(Ci, dtype, device)
    igg.update_halo(T, C, stream=stream)
    return T, C


def forward(T, Ci, nt, lam, dt, dx, dy, dz, split=(16, 2, 2), work=None, sr_seed=None, counter0=0,
            stream=None):
    """nt steps of the Fig. 1 time loop starting from T (valid halo).  Returns
    the tensor holding the final state, which is either T or `work` (the two
    buffers are swapped each step, as in the listing).  FP16 fields round
    their stores stochastically when sr_seed is given, with counter
    counter0 + step."""
    T2 = torch.empty_like(T) if work is None else work
    a, b = T, T2
    for it in range(nt):
        rnd = None
        if T.dtype == torch.float16 and sr_seed is not None:
            rnd = igg.rounding("stochastic", sr_seed, counter0 + it)
        igg.diffusion_step(b, a, Ci, lam, dt, dx, dy, dz, split=split, rnd=rnd, stream=stream)
        a, b = b, a
    return a


# --------------------------------------------------------------------------- checkpointing
def schedule_periodic(nt, every):
    """Snapshot steps of periodic checkpointing: 0, every, 2*every, ..."""
    return list(range(0, nt, every))


def schedule_sqrt(nt):
    """About sqrt(nt) evenly spaced snapshots."""
    return schedule_periodic(nt, max(1, int(round(math.sqrt(nt)))))


def binomial_reps(steps, snaps):
    """Smallest number r of forward sweeps per step such that binomial
    checkpointing with `snaps` snapshots covers `steps` steps: the least r with
    C(snaps + r, snaps) >= steps (Griewank and Walther, ACM TOMS 26, 2000)."""
    r = 0
    while math.comb(snaps + r, snaps) < steps:
        r += 1
    return r


def binomial_forward_cost(steps, snaps):
    """Forward steps spent by optimal binomial checkpointing to reverse
    `steps` steps with `snaps` snapshots (the initial state is held apart):
    r*steps - C(snaps + r, snaps - 1) + 1 with r from binomial_reps
    (Griewank, Optim. Methods Softw. 1, 1992), counting the first sweep."""
    if steps <= 1:
        return 0
    r = binomial_reps(steps, snaps)
    return r * steps - math.comb(snaps + r, snaps - 1) + 1


class _Revolve:
    """Binomial checkpointing plan (Griewank and Walther's Revolve idea):
    recursively reverse `steps` steps from a stored state with `snaps` free
    snapshot slots, advancing to the split point that the binomial
    coefficients make optimal, storing it, reversing the right part, then the
    left part with one slot fewer... and one slot returned."""

    def __init__(self, steps, snaps):
        self.steps, self.snaps = steps, snaps

    @staticmethod
    def split_point(steps, snaps):
        if snaps <= 0 or steps <= 1:
            return 0
        r = binomial_reps(steps, snaps)
        # largest forward advance for which the remaining parts stay within r sweeps
        best = max(1, min(steps - 1, math.comb(snaps + r - 1, snaps)))
        # the right part (steps - adv) must be reversible with snaps-1 slots and r sweeps,
        # the left part (adv) with snaps slots and r-1 sweeps
        adv = steps - min(steps - 1, math.comb(snaps - 1 + r, snaps - 1))
        adv = max(1, min(adv, best))
        return adv


def reverse_sweep_plan(nt, snaps):
    """Operations of binomial checkpointing for nt steps with `snaps` snapshot
    slots beside the initial state, as a list of ("advance", from, to),
    ("store", step), ("restore", step), ("adjoint", step), ("free", step).
    Used by tests to check validity and cost; the autograd driver executes
    the same plan."""
    ops = []

    def rev(start, end, slots):
        # state at `start` is available (stored); reverse steps start..end-1
        n = end - start
        if n == 0:
            return
        if n == 1:
            ops.append(("restore", start))
            ops.append(("adjoint", start))
            return
        if slots <= 0:
            # no free slot: recompute from start for every step
            for s in range(end - 1, start - 1, -1):
                ops.append(("restore", start))
                if s > start:
                    ops.append(("advance", start, s))
                ops.append(("adjoint", s))
            return
        adv = _Revolve.split_point(n, slots)
        mid = start + adv
        ops.append(("restore", start))
        ops.append(("advance", start, mid))
        ops.append(("store", mid))
        rev(mid, end, slots - 1)
        ops.append(("free", mid))
        rev(start, mid, slots)

    ops.append(("store", 0))
    rev(0, nt, snaps)
    return ops
