"""Virtual ranks: a dims[0] x dims[1] x dims[2] decomposition held as
separate blocks on one GPU, with the exchange between blocks.  Rank c's
block is the slice c*(n-ol) .. c*(n-ol)+n-1 of one block of the global size
N = dims*(n-ol)+ol (per dimension), so the halo update and the time loop on
the ranks must give that block's values bit for bit, and the global block
must match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, say  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def _global_n(n, ol, dims):
    return tuple(d * (m - o) + o for m, o, d in zip(n, ol, dims))


def _ranks(dims):
    return [(cx, cy, cz) for cz in range(dims[2]) for cy in range(dims[1]) for cx in range(dims[0])]


def _block(G, c, n, ol, extra=(0, 0, 0)):
    """Rank c's block of a global array G (z, y, x order); extra adds the
    staggered point of a face field per dimension."""
    sl = [slice(cd * (m - o), cd * (m - o) + m + e) for cd, m, o, e in zip(c, n, ol, extra)]
    return G[sl[2], sl[1], sl[0]]


CASES = [
    ((12, 10, 9), (2, 2, 2), (1, 1, 1), (2, 2, 2)),
    ((11, 9, 10), (3, 1, 2), (1, 0, 1), (2, 2, 3)),
    ((10, 12, 8), (1, 3, 1), (0, 1, 0), (3, 2, 2)),
    ((9, 9, 9), (2, 1, 1), (1, 1, 1), (2, 2, 2)),
]


@pytest.mark.parametrize("n,dims,periods,ol", CASES)
def test_halo_ranks_equal_global_halo(n, dims, periods, ol):
    """Each rank's halo planes that have a neighbour are overwritten with
    garbage; the exchange must restore the global block with its periodic
    halo (a cell-centred and a staggered field, FP64 and FP32)."""
    say("halo ranks", n, dims, periods, ol)
    N = _global_n(n, ol, dims)
    rng = np.random.default_rng(41)
    G = rng.uniform(-1, 1, (N[2], N[1], N[0]))
    Gq = rng.uniform(-1, 1, (N[2], N[1], N[0] + 1))  # x-face field
    ref = oracle.halo(G.copy(), ol, periods)
    refq = oracle.halo(Gq.copy(), (ol[0] + 1, ol[1], ol[2]), periods)
    with grid(n, periods, ol, dims=dims):
        ranks = _ranks(dims)
        per_rank = []
        for r, c in enumerate(ranks):
            assert igg.rank_coords(r) == c
            lo, hi = igg.neighbors(r)
            blocks = []
            for A, extra, dt in ((G, (0, 0, 0), torch.float64), (Gq, (1, 0, 0), torch.float32)):
                b = _block(A, c, n, ol, extra).copy()
                for d in range(3):
                    ax = 2 - d
                    if lo[d] >= 0:
                        np.moveaxis(b, ax, 0)[0] = 1e30
                    if hi[d] >= 0:
                        np.moveaxis(b, ax, 0)[-1] = 1e30
                blocks.append(dev(b, dt))
            per_rank.append(blocks)
        igg.update_halo_ranks(*per_rank)
        for r, c in enumerate(ranks):
            t, tq = per_rank[r]
            assert np.array_equal(host(t), _block(ref, c, n, ol)), r
            want = host(dev(_block(refq, c, n, ol, (1, 0, 0)), torch.float32))
            assert np.array_equal(host(tq), want), r


def _global_problem(N, periods, ol, seed):
    T0, Ci = synth.noisy_state_uniform_ci(N[0], N[1], N[2], seed=seed, noise=1e-2)
    oracle.halo(T0, ol, periods)
    oracle.halo(Ci, ol, periods)
    return T0, Ci


# rows of 72 points take the kernels of 4-point vectors: with x overlap 3 the
# second x rank's origin is odd (69), so its FP16 stochastic rounding takes
# the per-pair hash while the first rank's takes whole pairs per vector
@pytest.mark.parametrize("n,dims,periods,ol", CASES + [((70, 40, 36), (2, 2, 2), (1, 1, 1), (2, 2, 2)),
                                                      ((72, 40, 36), (2, 1, 1), (1, 1, 1), (3, 2, 2)),
                                                      ((72, 40, 36), (2, 2, 1), (1, 1, 1), (2, 2, 2))])
@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_step_ranks_equal_global_block(n, dims, periods, ol, dt_name):
    """nt steps on the ranks (split and unsplit) give the global block's
    nt steps bit for bit, halos included; FP64 also matches the oracle."""
    N = _global_n(n, ol, dims)
    T0, Ci = _global_problem(N, periods, ol, 43)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    nt = 5
    seed = 11 if dt_name == "f16" else None
    wdt = DT[dt_name]
    with grid(N, periods, ol):
        say("global block", N, dt_name)
        glob = host(diffusion.forward(dev(T0, wdt), dev(Ci, wdt), nt, 1.0, dt, dx, dx, dx, split=None,
                                      sr_seed=seed))
    if dt_name == "f64":
        ref = oracle.run(T0, Ci, nt, 1.0, dt, dx, dx, dx, ol=ol, periods=periods)
        assert np.max(np.abs(glob - ref)) <= 1e-12 * np.max(np.abs(ref))
    ranks = _ranks(dims)
    for split in [None, (4, 3, 3), (16, 2, 2)]:
        if split is not None and any(w < o for w, o in zip(split, ol)):
            continue
        with grid(n, periods, ol, dims=dims):
            say("step ranks", n, dims, periods, ol, dt_name, split)
            Ts = [dev(_block(T0, c, n, ol), wdt) for c in ranks]
            Cs = [dev(_block(Ci, c, n, ol), wdt) for c in ranks]
            Ws = [t.clone() for t in Ts]
            a, b = Ts, Ws
            for it in range(nt):
                rnd = igg.rounding("stochastic", seed, it) if seed is not None else None
                igg.diffusion_step_ranks(b, a, Cs, 1.0, dt, dx, dx, dx, split=split, rnd=rnd)
                a, b = b, a
            for r, c in enumerate(ranks):
                assert np.array_equal(host(a[r]), _block(glob, c, n, ol)), (split, r, c)


@pytest.mark.parametrize("n,dims,periods,ol", CASES)
@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_adjoint_ranks_equal_global_block(n, dims, periods, ol, dt_name):
    """Three adjoint steps on the ranks (split and unsplit) give the global
    block's lam_n bit for bit, halos included, and its gCi on every block's
    inner points."""
    N = _global_n(n, ol, dims)
    rng = np.random.default_rng(47)
    lam0, Tn, Ci = (rng.uniform(0.3, 0.9, (N[2], N[1], N[0])) for _ in range(3))
    for a in (lam0, Tn, Ci):
        oracle.halo(a, ol, periods)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    wdt = DT[dt_name]
    steps = 3
    with grid(N, periods, ol):
        say("adjoint global block", N, dt_name)
        lp, T, C = dev(lam0, wdt), dev(Tn, wdt), dev(Ci, wdt)
        g = torch.zeros_like(lp)
        for _ in range(steps):
            ln = lp.clone()
            igg.diffusion_step_adjoint(ln, lp, T, C, g, 1.0, dt, dx, dx, dx, split=None)
            lp = ln
        glob_l, glob_g = host(lp), host(g)
    ranks = _ranks(dims)
    for split in [None, (4, 3, 3)]:
        if split is not None and any(w < o for w, o in zip(split, ol)):
            continue
        with grid(n, periods, ol, dims=dims):
            say("adjoint ranks", n, dims, periods, ol, dt_name, split)
            lps = [dev(_block(lam0, c, n, ol), wdt) for c in ranks]
            Ts = [dev(_block(Tn, c, n, ol), wdt) for c in ranks]
            Cs = [dev(_block(Ci, c, n, ol), wdt) for c in ranks]
            gs = [torch.zeros_like(t) for t in lps]
            for _ in range(steps):
                lns = [t.clone() for t in lps]
                igg.diffusion_step_adjoint_ranks(lns, lps, Ts, Cs, gs, 1.0, dt, dx, dx, dx, split=split)
                lps = lns
            for r, c in enumerate(ranks):
                assert np.array_equal(host(lps[r]), _block(glob_l, c, n, ol)), (split, r)
                # gCi is accumulated on each block's inner points (its halo
                # stays as it was); those tile the global block's inner points
                assert np.array_equal(host(gs[r])[1:-1, 1:-1, 1:-1],
                                      _block(glob_g, c, n, ol)[1:-1, 1:-1, 1:-1]), (split, r)


@pytest.mark.parametrize("n,dims,periods,ol", CASES)
def test_flux_ranks_equal_global_block(n, dims, periods, ol):
    """The fused flux-form step on the ranks (split and unsplit): T and the
    three face fields equal the global block's bit for bit, halos included;
    then three flux-form adjoint steps give its lam_n (halos included) and
    gCi (inner points)."""
    N = _global_n(n, ol, dims)
    T0, Ci = _global_problem(N, periods, ol, 53)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    nt = 4
    fshape = [(N[2], N[1], N[0] + 1), (N[2], N[1] + 1, N[0]), (N[2] + 1, N[1], N[0])]
    extra = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    with grid(N, periods, ol):
        say("flux global block", N)
        T, C = dev(T0), dev(Ci)
        W = T.clone()
        q = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in fshape]
        for _ in range(nt):
            igg.diffusion_flux_step(W, T, C, *q, 1.0, dt, dx, dx, dx)
            T, W = W, T
        glob_T, glob_q = host(T), [host(x) for x in q]
        lp, g = T.clone(), torch.zeros_like(T)
        for _ in range(3):
            ln = lp.clone()
            igg.diffusion_flux_step_adjoint(ln, lp, T, C, g, 1.0, dt, dx, dx, dx)
            lp = ln
        glob_l, glob_g = host(lp), host(g)
    ranks = _ranks(dims)
    for split in [None, (4, 3, 3)]:
        if split is not None and any(w < o + 1 for w, o in zip(split, ol)):
            continue
        with grid(n, periods, ol, dims=dims):
            say("flux ranks", n, dims, periods, ol, split)
            Ts = [dev(_block(T0, c, n, ol)) for c in ranks]
            Cs = [dev(_block(Ci, c, n, ol)) for c in ranks]
            Ws = [t.clone() for t in Ts]
            qs = [[torch.zeros(tuple(m + e for m, e in zip((n[2], n[1], n[0]), reversed(ex))),
                               dtype=torch.float64, device="cuda") for ex in extra] for _ in ranks]
            a, b = Ts, Ws
            for _ in range(nt):
                igg.diffusion_flux_step_ranks(b, a, Cs, [x[0] for x in qs], [x[1] for x in qs], [x[2] for x in qs],
                                              1.0, dt, dx, dx, dx, split=split)
                a, b = b, a
            for r, c in enumerate(ranks):
                assert np.array_equal(host(a[r]), _block(glob_T, c, n, ol)), (split, r)
                for d in range(3):
                    assert np.array_equal(host(qs[r][d]), _block(glob_q[d], c, n, ol, extra[d])), (split, r, d)
            lps = [t.clone() for t in a]
            gs = [torch.zeros_like(t) for t in a]
            for _ in range(3):
                lns = [t.clone() for t in lps]
                igg.diffusion_flux_step_adjoint_ranks(lns, lps, a, Cs, gs, 1.0, dt, dx, dx, dx, split=split)
                lps = lns
            for r, c in enumerate(ranks):
                assert np.array_equal(host(lps[r]), _block(glob_l, c, n, ol)), (split, r)
                assert np.array_equal(host(gs[r])[1:-1, 1:-1, 1:-1],
                                      _block(glob_g, c, n, ol)[1:-1, 1:-1, 1:-1]), (split, r)


@pytest.mark.parametrize("n,dims,periods", [((12, 10, 9), (2, 2, 2), (1, 1, 1)), ((11, 9, 10), (3, 1, 2), (1, 0, 1)),
                                            ((40, 30, 24), (2, 1, 2), (1, 1, 1))])
def test_checkpointed_gradient_on_ranks_equals_global_block(n, dims, periods):
    """The checkpointed sweep over virtual ranks (snapshots every 3 steps)
    gives the global block's gradients bit for bit on every block's inner
    points, and its loss to the reduction order."""
    ol = (2, 2, 2)
    N = _global_n(n, ol, dims)
    rng = np.random.default_rng(59)
    T0, Ci, Tobs = (rng.uniform(0.3, 0.9, (N[2], N[1], N[0])) for _ in range(3))
    for a in (T0, Ci, Tobs):
        oracle.halo(a, ol, periods)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    nt = 8
    with grid(N, periods, ol):
        say("gradient global block", N)
        prob = diffusion.Problem(1.0, dt, dx, dx, dx, split=(4, 3, 3))
        L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt, ("periodic", 3))
        gT, gC = host(gT), host(gC)
    ranks = _ranks(dims)
    with grid(n, periods, ol, dims=dims):
        say("gradient ranks", n, dims, periods)
        prob = diffusion.RankProblem(1.0, dt, dx, dx, dx, split=(4, 3, 3))
        Lr, gTr, gCr, sw = diffusion.loss_and_grad_ranks([dev(_block(T0, c, n, ol)) for c in ranks],
                                                         [dev(_block(Ci, c, n, ol)) for c in ranks],
                                                         [dev(_block(Tobs, c, n, ol)) for c in ranks],
                                                         prob, nt, ("periodic", 3))
        assert sw.adjoints == nt
        for r, c in enumerate(ranks):
            for got, ref in ((gTr[r], gT), (gCr[r], gC)):
                assert np.array_equal(host(got)[1:-1, 1:-1, 1:-1], _block(ref, c, n, ol)[1:-1, 1:-1, 1:-1]), r
    assert abs(Lr - L) <= 1e-13 * L


def _grad_problem(N, periods, seed):
    ol = (2, 2, 2)
    rng = np.random.default_rng(seed)
    T0, Ci, Tobs = (rng.uniform(0.3, 0.9, (N[2], N[1], N[0])) for _ in range(3))
    for a in (T0, Ci, Tobs):
        oracle.halo(a, ol, periods)
    return T0, Ci, Tobs


@pytest.mark.parametrize("n,dims,periods,split", [((12, 10, 9), (2, 2, 2), (1, 1, 1), None),
                                                  ((11, 9, 10), (3, 1, 2), (1, 0, 1), (4, 3, 3)),
                                                  ((20, 16, 14), (2, 1, 2), (1, 1, 0), (4, 3, 3))])
def test_flux_checkpointed_gradient_on_ranks_equals_global_block(n, dims, periods, split):
    """The checkpointed sweep of the staggered flux form over virtual ranks
    (snapshots every 3 steps) gives the global block's gradients bit for bit
    on every block's inner points, and its loss to the reduction order."""
    ol = (2, 2, 2)
    N = _global_n(n, ol, dims)
    T0, Ci, Tobs = _grad_problem(N, periods, 61)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    nt = 7
    with grid(N, periods, ol):
        say("flux gradient global block", N, split)
        prob = diffusion.FluxProblem(1.0, dt, dx, dx, dx, split=split)
        L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt, ("periodic", 3))
        gT, gC = host(gT), host(gC)
    ranks = _ranks(dims)
    with grid(n, periods, ol, dims=dims):
        say("flux gradient ranks", n, dims, periods, split)
        prob = diffusion.FluxRankProblem(1.0, dt, dx, dx, dx, split=split)
        Lr, gTr, gCr, sw = diffusion.loss_and_grad_ranks([dev(_block(T0, c, n, ol)) for c in ranks],
                                                         [dev(_block(Ci, c, n, ol)) for c in ranks],
                                                         [dev(_block(Tobs, c, n, ol)) for c in ranks],
                                                         prob, nt, ("periodic", 3))
        assert sw.adjoints == nt
        for r, c in enumerate(ranks):
            for got, ref in ((gTr[r], gT), (gCr[r], gC)):
                assert np.array_equal(host(got)[1:-1, 1:-1, 1:-1], _block(ref, c, n, ol)[1:-1, 1:-1, 1:-1]), r
    assert abs(Lr - L) <= 1e-13 * L


@pytest.mark.parametrize("form", ["laplacian", "flux"])
@pytest.mark.parametrize("n,dims,periods", [((12, 10, 9), (2, 2, 2), (1, 1, 1)),
                                            ((11, 9, 10), (3, 1, 2), (1, 0, 1))])
def test_diffusion_solve_ranks_autograd_equals_global(n, dims, periods, form):
    """torch.autograd through DiffusionSolveRanks (loss over the blocks'
    inner points, written in torch) gives the global DiffusionSolve's
    T_nt and gradients bit for bit on every block's inner points."""
    ol = (2, 2, 2)
    N = _global_n(n, ol, dims)
    T0, Ci, Tobs = _grad_problem(N, periods, 67)
    dx = 1.0 / (N[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    nt = 6
    sched = ("binomial", 2)
    single = diffusion.Problem if form == "laplacian" else diffusion.FluxProblem
    multi = diffusion.RankProblem if form == "laplacian" else diffusion.FluxRankProblem
    split = (4, 3, 3)

    def loss(T, O):
        d = T[1:-1, 1:-1, 1:-1] - O[1:-1, 1:-1, 1:-1]
        return 0.5 * (d * d).sum()

    with grid(N, periods, ol):
        say("solve global block", form, N)
        T, C = dev(T0).requires_grad_(), dev(Ci).requires_grad_()
        out = diffusion.DiffusionSolve.apply(T, C, single(1.0, dt, dx, dx, dx, split=split), nt, sched)
        loss(out, dev(Tobs)).backward()
        g_out, gT, gC = host(out), host(T.grad), host(C.grad)
    ranks = _ranks(dims)
    with grid(n, periods, ol, dims=dims):
        say("solve ranks", form, n, dims, periods)
        Ts = [dev(_block(T0, c, n, ol)).requires_grad_() for c in ranks]
        Cs = [dev(_block(Ci, c, n, ol)).requires_grad_() for c in ranks]
        outs = diffusion.DiffusionSolveRanks.apply(multi(1.0, dt, dx, dx, dx, split=split), nt, sched, *Ts, *Cs)
        assert len(outs) == len(ranks)
        sum(loss(o, dev(_block(Tobs, c, n, ol))) for o, c in zip(outs, ranks)).backward()
        for r, c in enumerate(ranks):
            assert np.array_equal(host(outs[r]), _block(g_out, c, n, ol)), r
            for got, ref in ((Ts[r].grad, gT), (Cs[r].grad, gC)):
                assert np.array_equal(host(got), _block(ref, c, n, ol) * _inner_mask(n)), r


def _inner_mask(n):
    m = np.zeros((n[2], n[1], n[0]))
    m[1:-1, 1:-1, 1:-1] = 1.0
    return m
