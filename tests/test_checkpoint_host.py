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
