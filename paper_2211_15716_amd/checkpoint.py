"""Time-loop checkpointing schedules for the reverse (adjoint) sweep.

A schedule is a list of operations on states T_n of the time loop:
  ("restore", a)      make the stored state T_a current
  ("advance", a, b)   step the current state T_a forward to T_b
  ("store", b)        keep a copy of the current state T_b
  ("free", b)         drop the stored copy of T_b
  ("adjoint", n)      run the adjoint of step n (needs T_n current)
It starts with T_0 stored.  Everything up to the first adjoint operation is
the forward sweep (one more step from T_{nt-1} gives T_nt for the loss); the
rest is the reverse sweep.  Schedules:

  store_all      every state kept: no recomputation, nt snapshots;
  periodic(k)    snapshots every k steps; the reverse sweep recomputes one
                 segment at a time into a segment buffer of up to k states;
  sqrt           periodic with k = round(sqrt(nt));
  binomial(s)    optimal offline checkpointing with s snapshot slots (the
                 slot holding T_0 included), after Griewank, "Achieving
                 logarithmic growth of temporal and spatial complexity in
                 reverse automatic differentiation", Optim. Methods Softw. 1
                 (1992), and Griewank and Walther, "Algorithm 799: Revolve",
                 ACM TOMS 26 (2000): reverse l steps by advancing to a split
                 point chosen from the binomial numbers beta(s, t) = C(s+t, s),
                 storing it, reversing the right part with one slot fewer and
                 then the left part with the slot returned.
"""
import math


def beta(s, t):
    """Number of steps reversible with s snapshot slots when no step is
    advanced more than t times: C(s + t, s)."""
    if s < 0 or t < 0:
        return 0
    return math.comb(s + t, s)


def repetitions(l, s):
    """Smallest t with beta(s, t) >= l."""
    t = 0
    while beta(s, t) < l:
        t += 1
    return t


def binomial_advances(l, s):
    """Closed-form minimal number of forward steps to reverse l steps with s
    slots, the slot of T_0 included (Griewank 1992): t*l - beta(s+1, t-1)
    with t = repetitions(l, s); l(l-1)/2 for a single slot."""
    if l <= 1:
        return 0
    t = repetitions(l, s)
    return t * l - beta(s + 1, t - 1)


def _split(l, s):
    """Optimal first advance d for l steps and s slots, t = repetitions(l, s).
    The left part (d steps, s slots, already advanced once) must fit t-1
    repetitions and the right part (l-d steps, s-1 slots) t repetitions, and
    for the fewest total steps both must need all of them:
      max(l - beta(s-1, t), beta(s, t-2)) <= d <= min(beta(s, t-1), l - beta(s-1, t-1)).
    The smallest such d is taken."""
    t = repetitions(l, s)
    lo = max(1, l - beta(s - 1, t), beta(s, t - 2))
    hi = min(l - 1, beta(s, t - 1), l - beta(s - 1, t - 1))
    assert lo <= hi, (l, s, t)
    return lo


def binomial(nt, snaps):
    """Revolve-style schedule with `snaps` >= 1 slots (T_0 in one of them)."""
    if snaps < 1:
        raise ValueError("binomial checkpointing needs at least one slot")
    ops = []

    def rev(start, end, s):
        l = end - start
        if l == 1:
            ops.append(("restore", start))
            ops.append(("adjoint", start))
            return
        if s == 1:
            for n in range(end - 1, start - 1, -1):
                ops.append(("restore", start))
                if n > start:
                    ops.append(("advance", start, n))
                ops.append(("adjoint", n))
            return
        m = start + _split(l, s)
        ops.append(("restore", start))
        ops.append(("advance", start, m))
        ops.append(("store", m))
        rev(m, end, s - 1)
        ops.append(("free", m))
        rev(start, m, s)

    if nt > 0:
        rev(0, nt, snaps)
    return ops


def periodic(nt, every):
    """Snapshots at 0, every, 2*every, ...; each segment is recomputed into a
    buffer of its states before its adjoint steps run."""
    if every < 1:
        raise ValueError("checkpoint interval must be >= 1")
    ops = []
    starts = list(range(0, nt, every))
    # forward sweep: keep the segment starts
    for a, b in zip(starts[:-1], starts[1:]):
        ops.append(("restore", a))
        ops.append(("advance", a, b))
        ops.append(("store", b))
    for seg in range(len(starts) - 1, -1, -1):
        a = starts[seg]
        e = min(a + every, nt)
        ops.append(("restore", a))
        for n in range(a + 1, e):
            ops.append(("advance", n - 1, n))
            ops.append(("store", n))
        for n in range(e - 1, a - 1, -1):
            ops.append(("restore", n))
            ops.append(("adjoint", n))
            if n > a:
                ops.append(("free", n))
        if a != 0:
            ops.append(("free", a))
    return ops


def store_all(nt):
    return periodic(nt, nt) if nt > 0 else []


def sqrt_schedule(nt):
    return periodic(nt, max(1, int(round(math.sqrt(nt)))))


def make(kind, nt, arg=None):
    if kind == "store_all":
        return store_all(nt)
    if kind == "periodic":
        return periodic(nt, int(arg))
    if kind == "sqrt":
        return sqrt_schedule(nt)
    if kind == "binomial":
        return binomial(nt, int(arg))
    raise ValueError(kind)


def forward_part(ops):
    """Split a schedule into its forward sweep and reverse sweep."""
    for q, op in enumerate(ops):
        if op[0] == "adjoint":
            return ops[:q], ops[q:]
    return ops, []


def simulate(ops, nt):
    """Check a schedule on integer states; returns (advances, peak stored
    snapshots, adjoint order).  Raises if an adjoint step would see the
    wrong state or a restore finds nothing stored."""
    stored = {0}
    cur = 0
    advances = 0
    peak = 1
    order = []
    fwd, rev = forward_part(ops)
    for op in fwd:
        cur, advances = _apply(op, cur, stored, advances)
        peak = max(peak, len(stored))
    if nt > 0:
        assert cur == nt - 1, (cur, nt)
        advances += 1  # T_{nt-1} -> T_nt for the loss
    for op in rev:
        if op[0] == "adjoint":
            assert cur == op[1], (op, cur)
            order.append(op[1])
            continue
        cur, advances = _apply(op, cur, stored, advances)
        peak = max(peak, len(stored))
    assert order == list(range(nt - 1, -1, -1)), order
    return advances, peak, order


def _apply(op, cur, stored, advances):
    kind = op[0]
    if kind == "restore":
        assert op[1] in stored, op
        return op[1], advances
    if kind == "advance":
        assert cur == op[1], (op, cur)
        return op[2], advances + (op[2] - op[1])
    if kind == "store":
        assert cur == op[1], (op, cur)
        stored.add(op[1])
        return cur, advances
    if kind == "free":
        stored.discard(op[1])
        return cur, advances
    raise ValueError(op)
