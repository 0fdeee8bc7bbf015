"""Checkpointing schedules (host logic): every adjoint step sees the right
state, the binomial schedule spends the fewest forward steps -- equal to a
brute-force minimisation and to Griewank's closed form -- within its slots,
and running a schedule with the CPU oracle's step and adjoint reproduces the
store-all gradient bit for bit."""
import math
from functools import lru_cache

import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import checkpoint as ck
from paper_2211_15716_amd import synth


@lru_cache(None)
def _brute(l, s):
    """Fewest forward steps to reverse l steps from a stored start with s
    slots: try every first split point."""
    if l <= 1:
        return 0
    if s == 1:
        return l * (l - 1) // 2
    return min(d + _brute(l - d, s - 1) + _brute(d, s) for d in range(1, l))


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8])
def test_binomial_is_optimal_and_within_slots(s):
    for l in range(1, 80):
        adv, peak, _ = ck.simulate(ck.binomial(l, s), l)
        assert adv - 1 == _brute(l, s) == ck.binomial_advances(l, s), (l, s)
        assert peak <= s


def test_binomial_counts_known_values():
    # one slot: every state recomputed from T_0
    assert ck.binomial_advances(10, 1) == 45
    # enough slots for one sweep: beta(s, 1) = s + 1 steps need each step once
    for s in (2, 5, 9):
        assert ck.binomial_advances(s + 1, s) == s
    # the 200-step, 13-slot case of the inverse problem
    t = ck.repetitions(200, 13)
    assert math.comb(13 + t - 1, 13) < 200 <= math.comb(13 + t, 13)


@pytest.mark.parametrize("nt,k", [(1, 1), (7, 3), (16, 16), (200, 16), (100, 10), (13, 5)])
def test_periodic_schedule(nt, k):
    adv, peak, order = ck.simulate(ck.periodic(nt, k), nt)
    nseg = math.ceil(nt / k)
    last = nt - (nseg - 1) * k
    # the forward sweep (nt steps) runs through the last segment; every other
    # segment is recomputed once, its start excepted
    assert adv == nt + (nt - last) - (nseg - 1)
    assert peak <= nseg + k


def test_sqrt_and_store_all():
    adv, peak, _ = ck.simulate(ck.store_all(50), 50)
    assert adv == 50 and peak == 50
    adv, peak, _ = ck.simulate(ck.sqrt_schedule(100), 100)
    assert peak <= 10 + 10


def _run_schedule_on_oracle(ops, T0, Ci, Tobs, nt, lam, dt, d):
    """Execute a schedule with the oracle's step and adjoint (CPU)."""
    store = {0: T0.copy()}
    cur, cur_n = T0.copy(), 0
    fwd, rev = ck.forward_part(ops)

    def adv(a, b):
        nonlocal cur, cur_n
        assert cur_n == a
        for _ in range(a, b):
            nxt = oracle.step(cur, Ci, lam, dt, *d, out=cur.copy())
            oracle.halo(nxt)
            cur = nxt
        cur_n = b

    def do(op):
        nonlocal cur, cur_n
        if op[0] == "restore":
            cur, cur_n = store[op[1]].copy(), op[1]
        elif op[0] == "advance":
            adv(op[1], op[2])
        elif op[0] == "store":
            store[op[1]] = cur.copy()
        elif op[0] == "free":
            store.pop(op[1], None)

    for op in fwd:
        do(op)
    Tn = oracle.step(cur, Ci, lam, dt, *d, out=cur.copy())
    oracle.halo(Tn)
    lp = np.zeros_like(T0)
    oracle.inner(lp)[...] = oracle.inner(Tn) - oracle.inner(Tobs)
    oracle.halo(lp)
    g = np.zeros_like(T0)
    for op in rev:
        if op[0] == "adjoint":
            assert cur_n == op[1]
            ln = oracle.adjoint_step(lp, cur, Ci, g, lam, dt, *d)
            oracle.halo(ln)
            lp = ln
        else:
            do(op)
    return lp, g


@pytest.mark.parametrize("sched", [("periodic", 4), ("sqrt", None), ("binomial", 3), ("binomial", 1)])
def test_schedule_reproduces_store_all_gradient(sched):
    n, nt = 9, 13
    T0, Ci, Tobs = synth.uniform_fields(n, n, n, seed=40, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a)
    dx = 1.0 / (n - 1)
    d = (dx, dx, dx)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    _, gT, gC = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, *d)
    lp, g = _run_schedule_on_oracle(ck.make(sched[0], nt, sched[1]), T0, Ci, Tobs, nt, 1.0, dt, d)
    assert np.array_equal(oracle.inner(lp), oracle.inner(gT))
    assert np.array_equal(oracle.inner(g), oracle.inner(gC))


class _RecordingProblem:
    """A stand-in for the GPU problem, on CPU tensors: the step writes only
    the inner points (T2 = 0.5*T + Ci, halo planes untouched, like the halo
    planes of non-periodic dimensions) and checks that the buffer it writes
    carries T0's halo planes; the adjoint records the state it is given."""

    def __init__(self, T0):
        import torch
        self.mask = torch.ones_like(T0, dtype=torch.bool)
        self.mask[1:-1, 1:-1, 1:-1] = False
        self.halo = T0[self.mask].clone()
        self.seen = []

    def step(self, out, T, Ci, stream=None):
        assert out is not T
        assert bool((out[self.mask] == self.halo).all())
        out[1:-1, 1:-1, 1:-1] = 0.5 * T[1:-1, 1:-1, 1:-1] + Ci[1:-1, 1:-1, 1:-1]

    def adjoint(self, lam_n, lam_np1, Tn, Ci, gCi, stream=None):
        self.seen.append(Tn.clone())
        lam_n.copy_(lam_np1)


@pytest.mark.parametrize("sched", [("store_all",), ("periodic", 3), ("periodic", 16), ("sqrt",), ("binomial", 1),
                                   ("binomial", 2), ("binomial", 4)])
@pytest.mark.parametrize("nt", [0, 1, 2, 7, 20])
def test_sweep_executes_schedule_on_buffers(sched, nt):
    """The GPU driver's executor (Sweep, with snapshots written in place
    and freed buffers reused) run on CPU tensors: the forward result is the
    direct loop's, every adjoint step sees its state T_n, T0 is never
    written, the step count is the schedule's, and no more buffers are made
    than the schedule's peak number of snapshots."""
    torch = pytest.importorskip("torch")
    from paper_2211_15716_amd import diffusion
    rng = np.random.default_rng(nt)
    T0 = torch.from_numpy(rng.uniform(0.0, 1.0, (5, 6, 7)))
    Ci = torch.from_numpy(rng.uniform(0.0, 1.0, (5, 6, 7)))
    T0_copy = T0.clone()
    states = [T0.clone()]
    for _ in range(nt):
        nxt = states[-1].clone()
        nxt[1:-1, 1:-1, 1:-1] = 0.5 * states[-1][1:-1, 1:-1, 1:-1] + Ci[1:-1, 1:-1, 1:-1]
        states.append(nxt)
    prob = _RecordingProblem(T0)
    ops = ck.make(sched[0], nt, sched[1] if len(sched) > 1 else None)
    made = []
    real = diffusion._clone, diffusion._fresh_like, diffusion._zeros_like

    def counting(f):
        def g(x):
            y = f(x)
            made.append(y)
            return y
        return g

    # on CPU tensors the library's fills are replaced by torch's: a fresh
    # buffer is a copy (it must carry the non-periodic halo planes) and the
    # reverse sweep's zeroed buffers are torch zeros
    diffusion._clone = counting(real[0])
    diffusion._fresh_like = counting(real[0])
    diffusion._zeros_like = lambda x: diffusion._map(torch.zeros_like, x)
    try:
        sw = diffusion.Sweep(prob, Ci, T0, ops)
        out = sw.forward(nt)
        assert torch.equal(out, states[nt])
        sw.reverse(torch.zeros_like(T0))
    finally:
        diffusion._clone, diffusion._fresh_like, diffusion._zeros_like = real
    assert torch.equal(T0, T0_copy)
    assert len(prob.seen) == nt
    for q, seen in enumerate(prob.seen):
        assert torch.equal(seen, states[nt - 1 - q]), q
    assert sw.advances == sum(op[2] - op[1] for op in ops if op[0] == "advance") + (nt > 0)
    # two work buffers, the forward result, and at most peak-1 snapshot buffers
    assert len(made) <= 3 + sw.peak - 1


def test_hashed_fields_agree_between_host_and_torch():
    """The hashed input fields (made whole on the device, recomputed point by
    point on the host for the sampled parity checks of fields beyond 2^31
    points) agree bit for bit between torch and numpy, match the hash written
    out in plain Python integers, and fill [offset, offset + 1)."""
    torch = pytest.importorskip("torch")
    t = synth.hashed_field_torch(9, 7, 5, 23, 0.5, "cpu", planes=2)
    idx = np.arange(9 * 7 * 5).reshape(5, 7, 9)
    assert np.array_equal(t.numpy(), 0.5 + synth.hashed_uniform(idx, 23))

    def plain(v):
        for _ in range(2):
            v = (((v >> 16) ^ v) * 0x45D9F3B) % (1 << 32)
        return (v >> 16) ^ v

    big = [0, 1, 77, (1 << 31) - 1, 1 << 31, (1 << 31) + 12345, (1 << 32) - 1]
    want = [plain((i ^ 23) % (1 << 32)) / 2.0 ** 32 for i in big]
    assert np.array_equal(synth.hashed_uniform(big, 23), np.array(want))
    u = synth.hashed_uniform(np.arange(1 << 16), 5)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
