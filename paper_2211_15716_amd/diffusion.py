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
    buffers are swapped each step, as in the listing; a given `work` must
    hold T's halo planes in non-periodic dimensions).  FP16 fields round
    their stores stochastically when sr_seed is given, with counter
    counter0 + step."""
    # Fig. 1 starts the second buffer as a copy of the first: halo planes of
    # non-periodic dimensions are never written by the step, so both buffers
    # must carry them from the start
    T2 = T.clone() if work is None else work
    a, b = T, T2
    for it in range(nt):
        rnd = None
        if T.dtype == torch.float16 and sr_seed is not None:
            rnd = igg.rounding("stochastic", sr_seed, counter0 + it)
        igg.diffusion_step(b, a, Ci, lam, dt, dx, dy, dz, split=split, rnd=rnd, stream=stream)
        a, b = b, a
    return a


def forward_with(prob, T, Ci, nt, stream=None):
    """nt steps of `prob` (a Problem or FluxProblem) from T (valid halo),
    swapping two buffers as the Fig. 1 loop does; returns the final state."""
    a, b = T, T.clone()
    for _ in range(nt):
        prob.step(b, a, Ci, stream=stream)
        a, b = b, a
    return a


# --------------------------------------------------------------------------- adjoint sweep
class Problem:
    """Constants of one time loop: lam, dt (held fixed), spacings, split."""

    def __init__(self, lam, dt, dx, dy, dz, split=(16, 2, 2)):
        self.lam, self.dt, self.dx, self.dy, self.dz = lam, dt, dx, dy, dz
        self.split = split

    def step(self, out, T, Ci, stream=None):
        igg.diffusion_step(out, T, Ci, self.lam, self.dt, self.dx, self.dy, self.dz, split=self.split,
                           stream=stream)

    def adjoint(self, lam_n, lam_np1, Tn, Ci, gCi, stream=None):
        igg.diffusion_step_adjoint(lam_n, lam_np1, Tn, Ci, gCi, self.lam, self.dt, self.dx, self.dy, self.dz,
                                   split=self.split, stream=stream)


class FluxProblem:
    """The staggered flux form of the same time loop (Sec. 2 staggered grid)
    behind the interface Sweep uses: step(out, T, Ci) runs
    diffusion_flux_step with the face fluxes in work arrays (made on first
    use; `fluxes` holds the last step's), and adjoint(lam_n, lam_np1, Tn,
    Ci, gCi) runs diffusion_flux_step_adjoint, which forms the fluxes of
    step n from the state Tn."""

    def __init__(self, lam, dt, dx, dy, dz, split=None):
        self.lam, self.dt, self.dx, self.dy, self.dz = lam, dt, dx, dy, dz
        self.split = split
        self._q = None

    @staticmethod
    def face_arrays(T):
        """Zeroed face-flux arrays qx (nx+1 faces in x), qy, qz for a cell field T."""
        nz, ny, nx = T.shape
        shapes = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
        return [torch.zeros(s, dtype=T.dtype, device=T.device) for s in shapes]

    def _faces(self, T):
        if self._q is None:
            self._q = self.face_arrays(T)
        return self._q

    def step(self, out, T, Ci, stream=None):
        q = self._faces(T)
        igg.diffusion_flux_step(out, T, Ci, *q, self.lam, self.dt, self.dx, self.dy, self.dz, split=self.split,
                                stream=stream)

    @property
    def fluxes(self):
        """The face fluxes of the last step (qx, qy, qz)."""
        return self._q

    def adjoint(self, lam_n, lam_np1, Tn, Ci, gCi, stream=None):
        igg.diffusion_flux_step_adjoint(lam_n, lam_np1, Tn, Ci, gCi, self.lam, self.dt, self.dx, self.dy, self.dz,
                                        split=self.split, stream=stream)


class RankProblem(Problem):
    """The Laplacian time loop on a grid of several virtual ranks: states,
    Ci and gradients are lists with one block per rank, and the steps go
    through diffusion_step_ranks / diffusion_step_adjoint_ranks."""

    def step(self, out, T, Ci, stream=None):
        igg.diffusion_step_ranks(out, T, Ci, self.lam, self.dt, self.dx, self.dy, self.dz, split=self.split,
                                 stream=stream)

    def adjoint(self, lam_n, lam_np1, Tn, Ci, gCi, stream=None):
        igg.diffusion_step_adjoint_ranks(lam_n, lam_np1, Tn, Ci, gCi, self.lam, self.dt, self.dx, self.dy, self.dz,
                                         split=self.split, stream=stream)


class FluxRankProblem(FluxProblem):
    """The staggered flux form on a grid of virtual ranks: states, Ci and
    gradients are lists with one block per rank, the face fluxes one
    (qx, qy, qz) triple per rank (`fluxes`), and the steps go through
    diffusion_flux_step_ranks / diffusion_flux_step_adjoint_ranks."""

    def _faces(self, Ts):
        if self._q is None:
            self._q = [self.face_arrays(T) for T in Ts]
        return self._q

    def step(self, out, T, Ci, stream=None):
        q = self._faces(T)
        igg.diffusion_flux_step_ranks(out, T, Ci, [x[0] for x in q], [x[1] for x in q], [x[2] for x in q],
                                      self.lam, self.dt, self.dx, self.dy, self.dz, split=self.split, stream=stream)

    def adjoint(self, lam_n, lam_np1, Tn, Ci, gCi, stream=None):
        igg.diffusion_flux_step_adjoint_ranks(lam_n, lam_np1, Tn, Ci, gCi, self.lam, self.dt, self.dx, self.dy,
                                              self.dz, split=self.split, stream=stream)


# states are tensors, or lists of per-rank blocks on a grid of virtual ranks
def _map(f, x):
    return [f(t) for t in x] if isinstance(x, (list, tuple)) else f(x)


def _clone(x):
    return _map(torch.clone, x)


def _zeros_like(x):
    """Zero-filled buffers like x (filled by the library)."""
    def one(t):
        y = torch.empty_like(t)
        igg.adjoint_seed(y, halo=False)
        return y
    return _map(one, x)


def _restrict(t, halo):
    """A new buffer with t's inner points and a zero halo, then (halo set) the
    halo update: the library's adjoint seed without T_obs."""
    y = torch.empty_like(t)
    igg.adjoint_seed(y, t, halo=halo)
    return y


def _fresh_like(x):
    """New buffers for a step's output: a step writes every inner point and
    the halo planes of periodic dimensions, so on a fully periodic grid an
    uninitialised buffer will do; otherwise a copy of x carries the halo
    planes of the non-periodic dimensions, which are the same in every
    state."""
    if all(igg.topology()["periods"]):
        return _map(torch.empty_like, x)
    return _clone(x)


def _copy_(dst, src):
    if isinstance(dst, (list, tuple)):
        for d, s_ in zip(dst, src):
            d.copy_(s_)
    else:
        dst.copy_(src)


def _fuse_stores(ops):
    """Merge ("advance", a, b) followed by ("store", b) into
    ("advance_store", a, b): the last step then writes the snapshot itself
    instead of a work buffer that is copied afterwards."""
    out = []
    for op in ops:
        if op[0] == "store" and out and out[-1][0] == "advance" and out[-1][2] == op[1] and op[1] > out[-1][1]:
            out[-1] = ("advance_store", out[-1][1], op[1])
        else:
            out.append(op)
    return out


class Sweep:
    """Runs a checkpointing schedule (paper_2211_15716_amd.checkpoint) on the
    GPU.  Snapshots are device tensors (lists of per-rank blocks with a
    RankProblem); the current state is either a snapshot (read only) or one
    of two work buffers, so advancing never overwrites a snapshot.  A state
    that is stored right after it is computed is computed into its snapshot
    buffer directly, which is a freed snapshot's buffer when one is free (its
    halo planes in non-periodic dimensions hold T0's, which no step writes).
    Counts forward and adjoint steps."""

    def __init__(self, prob, Ci, T0, ops):
        self.p, self.Ci, self.ops = prob, Ci, ops
        self.store = {0: T0}
        self.work = [_clone(T0), _clone(T0)]  # halo planes of non-periodic dimensions
        self.pool = []  # buffers of freed snapshots
        self.cur, self.cur_n = T0, 0
        self.advances = 0
        self.adjoints = 0
        self.peak = 1
        self.fwd, self.rev = _split_ops(_fuse_stores(ops))

    def _advance(self, a, b):
        assert self.cur_n == a, (a, self.cur_n)
        for _ in range(a, b):
            dst = self.work[0] if self.cur is not self.work[0] else self.work[1]
            self.p.step(dst, self.cur, self.Ci)
            self.cur = dst
            self.advances += 1
        self.cur_n = b

    def _do(self, op):
        kind = op[0]
        if kind == "restore":
            self.cur, self.cur_n = self.store[op[1]], op[1]
        elif kind == "advance":
            self._advance(op[1], op[2])
        elif kind == "advance_store":
            a, b = op[1], op[2]
            self._advance(a, b - 1)
            dst = None
            for q, buf in enumerate(self.pool):
                if buf is not self.cur:
                    dst = self.pool.pop(q)
                    break
            if dst is None:
                dst = _fresh_like(self.cur)
            self.p.step(dst, self.cur, self.Ci)
            self.advances += 1
            self.cur, self.cur_n = dst, b
            self.store[b] = dst
            self.peak = max(self.peak, len(self.store))
        elif kind == "store":
            assert self.cur_n == op[1]
            self.store[op[1]] = _clone(self.cur)
            self.peak = max(self.peak, len(self.store))
        elif kind == "free":
            if op[1] != 0:  # T0 is the caller's tensor
                self.pool.append(self.store.pop(op[1]))
        else:
            raise ValueError(op)

    def forward(self, nt):
        """The forward sweep; returns T_nt (a new tensor)."""
        for op in self.fwd:
            self._do(op)
        if nt == 0:
            return _clone(self.cur)
        out = _fresh_like(self.cur)  # carries the non-periodic halo planes
        self.p.step(out, self.cur, self.Ci)
        self.advances += 1
        return out

    def reverse(self, lam_nt):
        """The reverse sweep from lam_nt = dLoss/dT_nt (valid halo); returns
        (dLoss/dT_0, dLoss/dCi) with the Ci gradient on the inner points."""
        lp = lam_nt
        # lambda lives on the unique points: its halo planes in non-periodic
        # dimensions stay zero (the adjoint steps never write them)
        ln = _zeros_like(lp)
        gCi = _zeros_like(lp)
        for op in self.rev:
            if op[0] == "adjoint":
                assert self.cur_n == op[1], (op, self.cur_n)
                self.p.adjoint(ln, lp, self.cur, self.Ci, gCi)
                lp, ln = ln, lp
                self.adjoints += 1
            else:
                self._do(op)
        return lp, gCi


def checkpoint_ops(kind, nt, arg=None):
    """Schedule of paper_2211_15716_amd.checkpoint by name."""
    from . import checkpoint
    return checkpoint.make(kind, nt, arg)


def _split_ops(ops):
    for q, op in enumerate(ops):
        if op[0] == "adjoint":
            return ops[:q], ops[q:]
    return ops, []


def _inner_only(t):
    """t's inner points with a zero halo (by the library)."""
    return _restrict(t.contiguous(), False)


class DiffusionSolve(torch.autograd.Function):
    """T_nt = nt steps of the Fig. 1 time loop from T0 with heat-capacity
    inverse Ci; differentiable in T0 and Ci by the hand-written adjoint
    kernels, with time-loop checkpointing.

    forward(T0, Ci, prob, nt, schedule) -- schedule is ("store_all",),
    ("periodic", k), ("sqrt",) or ("binomial", slots).  T0 and Ci must carry
    valid halos.  The gradients returned are zero on halo points: the loss
    may only depend on the unique (inner) points, and the incoming gradient
    is restricted to them and then given the periodic halo."""

    @staticmethod
    def forward(ctx, T0, Ci, prob, nt, schedule=("store_all",)):
        from . import checkpoint
        ops = checkpoint.make(schedule[0], nt, schedule[1] if len(schedule) > 1 else None)
        sweep = Sweep(prob, Ci, T0.detach(), ops)
        out = sweep.forward(nt)
        ctx.sweep = sweep
        ctx.nt = nt
        return out

    @staticmethod
    def backward(ctx, g):
        sweep = ctx.sweep
        lam_nt = _restrict(g.contiguous(), True)
        gT0, gCi = sweep.reverse(lam_nt)
        ctx.sweep = None
        return _inner_only(gT0), _inner_only(gCi), None, None, None


def _need_unit_overlaps(what):
    # with overlaps of 2 the blocks' inner points tile the global grid's
    # unique points, so a loss over every block's inner points counts each
    # unique point once
    if tuple(igg.topology()["overlaps"]) != (2, 2, 2):
        raise ValueError(what + " needs overlaps (2, 2, 2)")


class DiffusionSolveRanks(torch.autograd.Function):
    """DiffusionSolve on a grid of virtual ranks.

    apply(prob, nt, schedule, *blocks) -- blocks are the P blocks of T0
    followed by the P blocks of Ci (P = igg.nranks(), rank order), each with
    a valid halo; prob is a RankProblem or FluxRankProblem.  Returns the P
    blocks of T_nt.  The gradients (P blocks of dL/dT0, then P of dL/dCi)
    are zero on halo points: the loss may only depend on the blocks' inner
    points, which tile the global unique points (overlaps of 2 only)."""

    @staticmethod
    def forward(ctx, prob, nt, schedule, *blocks):
        from . import checkpoint
        P = igg.nranks()
        if len(blocks) != 2 * P:
            raise ValueError(f"expected {2 * P} blocks (T0 and Ci of {P} ranks), got {len(blocks)}")
        _need_unit_overlaps("DiffusionSolveRanks")
        ops = checkpoint.make(schedule[0], nt, schedule[1] if len(schedule) > 1 else None)
        sweep = Sweep(prob, [b.detach() for b in blocks[P:]], [b.detach() for b in blocks[:P]], ops)
        out = sweep.forward(nt)
        ctx.sweep = sweep
        return tuple(out)

    @staticmethod
    def backward(ctx, *gs):
        sweep = ctx.sweep
        lam_nt = [_restrict(g.contiguous(), False) for g in gs]
        igg.update_halo_ranks(*[(t,) for t in lam_nt])
        gT0, gCi = sweep.reverse(lam_nt)
        ctx.sweep = None
        return (None, None, None, *[_inner_only(t) for t in gT0], *[_inner_only(t) for t in gCi])


def loss_and_grad(T0, Ci, T_obs, prob, nt, schedule=("store_all",)):
    """0.5*||T_nt - T_obs||^2 over the unique points (FP64 reduction on the
    GPU) and its gradients (dL/dT0, dL/dCi), by DiffusionSolve."""
    from . import checkpoint
    ops = checkpoint.make(schedule[0], nt, schedule[1] if len(schedule) > 1 else None)
    sweep = Sweep(prob, Ci, T0, ops)
    Tnt = sweep.forward(nt)
    # the seed lam_nt = T_nt - T_obs (inner points, halo updated) and the loss
    # in one library call
    lam_nt = torch.empty_like(Tnt)
    L = igg.adjoint_seed(lam_nt, Tnt, T_obs, halo=True, loss=True)
    gT0, gCi = sweep.reverse(lam_nt)
    return L, _inner_only(gT0), _inner_only(gCi), sweep


def loss_and_grad_ranks(T0s, Cis, T_obs_s, prob, nt, schedule=("store_all",)):
    """loss_and_grad on a grid of virtual ranks (lists of per-rank blocks,
    prob a RankProblem or FluxRankProblem).  The blocks' inner points tile
    the global grid's unique points when the overlaps are 2, so the loss is
    the sum of the blocks' FP64 sums; other overlaps are refused."""
    from . import checkpoint
    _need_unit_overlaps("loss_and_grad_ranks")
    ops = checkpoint.make(schedule[0], nt, schedule[1] if len(schedule) > 1 else None)
    sweep = Sweep(prob, Cis, T0s, ops)
    Tnt = sweep.forward(nt)
    lam_nt = [torch.empty_like(a) for a in Tnt]
    L = sum(igg.adjoint_seed(lt, a, b, halo=False, loss=True) for lt, a, b in zip(lam_nt, Tnt, T_obs_s))
    igg.update_halo_ranks(*[(t,) for t in lam_nt])
    gT0, gCi = sweep.reverse(lam_nt)
    return L, [_inner_only(t) for t in gT0], [_inner_only(t) for t in gCi], sweep


# --------------------------------------------------------------------------- graph capture
class StepGraph:
    """A HIP graph holding 2*pairs consecutive diffusion steps T -> T2 -> T,
    for grids small enough that launch latency dominates (each step is a
    handful of short launches on two streams).  Replaying it advances the
    state held in T by 2*pairs steps, with the same bits as the eager calls.

    The step's fork and join events make it capturable across the helper
    stream.  The library's device resources are created before capture (the
    halo update of T below is idempotent: T carries a valid halo), since
    nothing may be allocated while a graph is being captured."""

    def __init__(self, T, T2, Ci, lam, dt, dx, dy, dz, split=(16, 2, 2), pairs=1):
        self.T, self.T2, self.Ci = T, T2, Ci
        igg.update_halo(T)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(pairs):
                igg.diffusion_step(T2, T, Ci, lam, dt, dx, dy, dz, split=split)
                igg.diffusion_step(T, T2, Ci, lam, dt, dx, dy, dz, split=split)
        self.steps = 2 * pairs

    def replay(self):
        self.graph.replay()
