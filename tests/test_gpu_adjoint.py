"""Adjoint sweep on the GPU: checkpointed equals store-all bit for bit,
parity with the oracle's gradient, the autograd path, the dot-product test,
central finite differences, and the 256^3 inverse-problem configuration."""
import math

import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, inner, say  # noqa: E402


def _fields(n, seed):
    nx, ny, nz = n
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=seed, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a)
    return T0, Ci, Tobs


@pytest.mark.parametrize("split", [(16, 2, 2), None])
def test_checkpointed_equals_store_all_and_oracle(split):
    say("checkpointed adjoint", split)
    n = (40, 34, 30)
    nt = 17
    T0, Ci, Tobs = _fields(n, 51)
    dx, dy, dz = 1 / 39, 1 / 33, 1 / 29
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    with grid(n):
        prob = diffusion.Problem(1.0, dt, dx, dy, dz, split=split)
        T, C, O = dev(T0), dev(Ci), dev(Tobs)
        res = {}
        for sched in [("store_all",), ("periodic", 4), ("sqrt",), ("binomial", 3), ("binomial", 1)]:
            L, gT, gC, sw = diffusion.loss_and_grad(T, C, O, prob, nt, sched)
            res[sched] = (L, host(gT), host(gC), sw.advances)
        L0, gT0, gC0, adv0 = res[("store_all",)]
        assert adv0 == nt
        for sched, (L, gT, gC, adv) in res.items():
            assert L == L0 and np.array_equal(gT, gT0) and np.array_equal(gC, gC0), sched
    assert abs(L0 - L_ref) <= 1e-12 * L_ref
    assert np.max(np.abs(inner(gT0) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC0) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


@pytest.mark.parametrize("split", [None, (16, 2, 2)])
def test_adjoint_multi_tile_matches_oracle(split):
    """A grid spanning several x and y tiles and z chunks of the adjoint
    kernel, with ragged tails."""
    say("adjoint multi-tile", split)
    n = (150, 60, 45)
    nt = 6
    T0, Ci, Tobs = _fields(n, 56)
    dx, dy, dz = 1 / 149, 1 / 59, 1 / 44
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    with grid(n):
        prob = diffusion.Problem(1.0, dt, dx, dy, dz, split=split)
        L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt)
        gT, gC = host(gT), host(gC)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


@pytest.mark.parametrize("n", [(40, 34, 30), (150, 60, 45)])
def test_adjoint_box_kernel_and_zmarch_paths_equal(n):
    """The adjoint's small-region box kernel and its z-march kernel give the
    same bits."""
    say("adjoint box vs zmarch", n)
    nt = 5
    T0, Ci, Tobs = _fields(n, 57)
    dx = 1 / (n[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    res = []
    for zmin in (None, 0):
        with grid(n, zmarch_min=zmin):
            prob = diffusion.Problem(1.0, dt, dx, dx, dx)
            L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt)
            res.append((L, host(gT), host(gC)))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])


def test_adjoint_schedules_and_x_exchange_forms_equal(monkeypatch):
    """The adjoint sweep under every schedule and both x-exchange forms (x
    halo of lam_n stored by the adjoint kernels, or a separate x pass) gives
    the same loss and gradients, bit for bit, and matches the oracle; the
    one-launch form (schedule 3, where the kernel also stores the y and z
    halo of lam_n) on the z-march and on the box kernels."""
    n = (70, 40, 36)
    nt = 6
    T0, Ci, Tobs = _fields(n, 58)
    dx = 1 / 69
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dx, dx)
    res = []
    combos = [(sched, xform, 0) for sched in ("1", "0", "2", "3") for xform in ("fused", "halo")]
    combos.append(("3", "fused", None))  # the box kernels of small regions
    for sched, xform, zmin in combos:
        monkeypatch.setenv("IGG_SCHEDULE", sched)
        monkeypatch.setenv("IGG_X_EXCHANGE", xform)
        with grid(n, zmarch_min=zmin):
            for split in [(16, 2, 2), None]:
                say("adjoint schedule", sched, xform, zmin, split)
                prob = diffusion.Problem(1.0, dt, dx, dx, dx, split=split)
                L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt)
                res.append((L, host(gT), host(gC)))
    for L, gT, gC in res[1:]:
        assert L == res[0][0] and np.array_equal(gT, res[0][1]) and np.array_equal(gC, res[0][2])
    L, gT, gC = res[0]
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


@pytest.mark.parametrize("periods", [(1, 0, 1), (0, 0, 0), (0, 1, 1)])
def test_checkpointed_gradient_non_periodic_matches_oracle(periods):
    """Non-periodic dimensions: the boundary planes are fixed inputs, the
    adjoint's halo there is zero; every schedule gives the oracle's loss and
    gradients."""
    say("non-periodic gradient", periods)
    n = (40, 34, 30)
    nt = 9
    T0, Ci, Tobs = synth.uniform_fields(*n, seed=63, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a, (2, 2, 2), periods)
    dx = 1 / 39
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dx, dx, periods=periods)
    with grid(n, periods):
        for split in (None, (16, 2, 2)):
            prob = diffusion.Problem(1.0, dt, dx, dx, dx, split=split)
            for sched in [("store_all",), ("periodic", 4), ("binomial", 2)]:
                L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt, sched)
                gT, gC = host(gT), host(gC)
                assert abs(L - L_ref) <= 1e-12 * L_ref
                assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref))), sched
                assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref))), sched


@pytest.mark.parametrize("ol", [(3, 3, 3), (2, 3, 4)])
@pytest.mark.parametrize("zmin", [0, None])
def test_checkpointed_gradient_wider_overlaps_matches_oracle(ol, zmin):
    """Periodic grid with overlaps above 2: on one rank the boundary-first
    adjoint fills the y/z halo of lambda from the images of its halo points
    (rows and planes ol-1 and n-ol) as it stores them, in the z-march
    (zmin 0) and the small-grid kernels (zmin None); every schedule gives
    the oracle's loss and gradients."""
    say("wider-overlap gradient", ol, zmin)
    n = (40, 34, 30)
    nt = 9
    T0, Ci, Tobs = synth.uniform_fields(*n, seed=67, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a, ol, (1, 1, 1))
    dx = 1 / 39
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dx, dx, ol=ol)
    with grid(n, overlaps=ol, zmarch_min=zmin):
        for split in (None, (16, 4, 4)):
            prob = diffusion.Problem(1.0, dt, dx, dx, dx, split=split)
            for sched in [("store_all",), ("periodic", 4)]:
                L, gT, gC, _ = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt, sched)
                gT, gC = host(gT), host(gC)
                assert abs(L - L_ref) <= 1e-12 * L_ref
                assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref))), sched
                assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref))), sched


def test_autograd_function_matches_sweep():
    say("autograd")
    n = (36, 30, 28)
    nt = 9
    T0, Ci, Tobs = _fields(n, 52)
    dx = 1 / 35
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    with grid(n):
        prob = diffusion.Problem(1.0, dt, dx, dx, dx)
        T, C, O = dev(T0), dev(Ci), dev(Tobs)
        L, gT, gC, _ = diffusion.loss_and_grad(T, C, O, prob, nt, ("binomial", 4))
        Ta, Ca = T.clone().requires_grad_(True), C.clone().requires_grad_(True)
        out = diffusion.DiffusionSolve.apply(Ta, Ca, prob, nt, ("periodic", 3))
        r = (out - O)[1:-1, 1:-1, 1:-1]
        loss = 0.5 * (r * r).sum()
        loss.backward()
        assert abs(loss.item() - L) <= 1e-13 * L
        assert torch.equal(Ta.grad, gT) and torch.equal(Ca.grad, gC)


def test_dot_product_on_gpu():
    """<J d, y> = <d, J^T y> for the map T0 -> T_nt (FP64 reductions)."""
    say("dot product")
    n = (48, 40, 36)
    nt = 12
    d0, Ci, y = _fields(n, 53)
    dx = 1 / 47
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    with grid(n):
        prob = diffusion.Problem(1.0, dt, dx, dx, dx)
        d, C, Y = dev(d0), dev(Ci), dev(y)
        Jd = diffusion.forward(d.clone(), C, nt, 1.0, dt, dx, dx, dx)
        lam = torch.zeros_like(Y)
        lam[1:-1, 1:-1, 1:-1] = Y[1:-1, 1:-1, 1:-1]
        igg.update_halo(lam)
        sw = diffusion.Sweep(prob, C, d, diffusion.checkpoint_ops("store_all", nt))
        sw.forward(nt)
        JTy, _ = sw.reverse(lam)
        lhs = igg.reduce(igg.RED_DOT, Jd, Y)
        rhs = igg.reduce(igg.RED_DOT, d, JTy)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _central(prob, T, C, O, nt, which, vox, h):
    """(L(x + h e) - L(x - h e)) / 2h along one unique voxel, the loss
    difference formed as a dot product of the pointwise state differences
    (so the unchanged points cancel exactly)."""
    k, j, i = vox
    outs = []
    for sgn in (+1, -1):
        Cp, Tp = C.clone(), T.clone()
        if which == "Ci":
            Cp[k, j, i] += sgn * h
            igg.update_halo(Cp)
        else:
            Tp[k, j, i] += sgn * h
            igg.update_halo(Tp)
        outs.append(diffusion.forward(Tp, Cp, nt, prob.lam, prob.dt, prob.dx, prob.dy, prob.dz,
                                      split=prob.split))
    diff = outs[0] - outs[1]
    mid = 0.5 * (outs[0] + outs[1]) - O
    return igg.reduce(igg.RED_DOT, diff, mid) / (2 * h)


def _fd_check(prob, T, C, O, nt, gC, gT, voxels, hrel=1e-2, hT=1e-3):
    """Finite-difference check at the given inner voxels.  L is quadratic in
    T0, so its central difference is exact up to rounding; in Ci it is a
    polynomial of degree nt, so the central difference is Richardson
    extrapolated from steps h and h/2, cancelling the h^2 error term.  The
    Ci step is 1e-2*Ci: the loss difference of two FP64 runs carries
    rounding noise near 1e-17 absolute, and most voxels' gradients are small,
    so a smaller step would measure that noise rather than the gradient.
    Relative error where |g| >= 1e-3 max|g|, else absolute over max|g|."""
    gmax_c = torch.max(torch.abs(gC)).item()
    gmax_t = torch.max(torch.abs(gT)).item()
    worst = 0.0
    for (k, j, i) in voxels:
        for which in ("Ci", "T0"):
            if which == "Ci":
                h = hrel * C[k, j, i].item()
                f1 = _central(prob, T, C, O, nt, which, (k, j, i), h)
                f2 = _central(prob, T, C, O, nt, which, (k, j, i), h / 2)
                fd = (4.0 * f2 - f1) / 3.0
            else:
                fd = _central(prob, T, C, O, nt, which, (k, j, i), hT)
            g = (gC if which == "Ci" else gT)[k, j, i].item()
            gmax = gmax_c if which == "Ci" else gmax_t
            if abs(g) >= 1e-3 * gmax:
                err = abs(fd - g) / abs(g)
            else:
                err = abs(fd - g) / gmax
            worst = max(worst, err)
    return worst


def test_gradient_matches_central_differences_small():
    say("FD small")
    n = (30, 26, 22)
    nt = 10
    T0, Ci, Tobs = _fields(n, 54)
    dx = 1 / 29
    dt = oracle.time_step(dx, dx, dx, 1.0, 1.0)
    rng = np.random.default_rng(5)
    vox = [(int(rng.integers(1, 21)), int(rng.integers(1, 25)), int(rng.integers(1, 29))) for _ in range(6)]
    with grid(n):
        prob = diffusion.Problem(1.0, dt, dx, dx, dx)
        T, C, O = dev(T0), dev(Ci), dev(Tobs)
        _, gT, gC, _ = diffusion.loss_and_grad(T, C, O, prob, nt, ("periodic", 4))
        worst = _fd_check(prob, T, C, O, nt, gC, gT, vox)
    assert worst <= 1e-6, worst


def test_inverse_problem_256_fd_20_voxels():
    """256^3 FP64, nt=200, snapshots every 16: T_obs from Ci_true (sine),
    guess Ci = 0.5, dt fixed from max(Ci_true); dL/dCi and dL/dT0 checked
    against central differences on 20 random unique voxels."""
    say("inverse 256^3 nt=200")
    w = synth.workload("c4_256_inverse", seed=0)
    n = (w["nx"], w["ny"], w["nz"])
    nt = w["nt"]
    with grid(n):
        T, Ctrue = diffusion.prepare_fields(w["T0"], w["Ci"])
        dt = igg.diffusion_dt(Ctrue, w["lam"], w["dx"], w["dy"], w["dz"])
        prob = diffusion.Problem(w["lam"], dt, w["dx"], w["dy"], w["dz"])
        O = diffusion.forward(T.clone(), Ctrue, nt, prob.lam, dt, prob.dx, prob.dy, prob.dz)
        C = torch.full_like(T, 0.5)
        L, gT, gC, sw = diffusion.loss_and_grad(T, C, O, prob, nt, ("periodic", 16))
        assert sw.adjoints == nt and L > 0
        rng = np.random.default_rng(0)
        vox = [tuple(int(v) for v in rng.integers(1, 255, size=3)) for _ in range(20)]
        worst = _fd_check(prob, T, C, O, nt, gC, gT, vox)
    assert worst <= 1e-6, worst


def test_fp32_adjoint_close_to_fp64():
    say("fp32 adjoint")
    n = (40, 36, 32)
    nt = 10
    T0, Ci, Tobs = _fields(n, 55)
    dx = 1 / 39
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    with grid(n):
        for prob in (diffusion.Problem(1.0, dt, dx, dx, dx), diffusion.FluxProblem(1.0, dt, dx, dx, dx),
                     diffusion.FluxProblem(1.0, dt, dx, dx, dx, split=(16, 3, 3))):
            say("fp32 adjoint", type(prob).__name__, prob.split)
            r64 = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt)
            prob32 = type(prob)(1.0, dt, dx, dx, dx, split=prob.split)
            r32 = diffusion.loss_and_grad(dev(T0, torch.float32), dev(Ci, torch.float32),
                                          dev(Tobs, torch.float32), prob32, nt)
            for a, b in ((r64[1], r32[1]), (r64[2], r32[2])):
                err = torch.max(torch.abs(a - b.double())).item() / torch.max(torch.abs(a)).item()
                assert err <= 1e-5, err


def test_flux_form_checkpointed_adjoint_matches_oracle():
    """The flux form through the checkpointed sweep (the adjoint forms the
    fluxes from the stored or recomputed states): every schedule and split
    gives the store-all loss and gradients bit for bit, and they match the
    oracle's flux-form gradient."""
    say("flux checkpointed adjoint")
    n = (34, 28, 24)
    nx, ny, nz = n
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=62, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a)
    d = (1 / 33, 1 / 27, 1 / 23)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 11
    L_ref, gT_ref, gC_ref = oracle.flux_gradient(T0, Ci, Tobs, nt, 1.0, dt, *d)
    with grid(n):
        res = {}
        for split in (None, (16, 3, 3)):
            prob = diffusion.FluxProblem(1.0, dt, *d, split=split)
            for sched in [("store_all",), ("sqrt",), ("periodic", 4), ("binomial", 3)]:
                L, gT, gC, sw = diffusion.loss_and_grad(dev(T0), dev(Ci), dev(Tobs), prob, nt, sched)
                res[(split,) + sched] = (L, host(gT), host(gC))
                assert sw.adjoints == nt
    L0, gT0, gC0 = res[(None, "store_all")]
    for sched, (L, gT, gC) in res.items():
        assert L == L0 and np.array_equal(gT, gT0) and np.array_equal(gC, gC0), sched
    assert abs(L0 - L_ref) <= 1e-12 * L_ref
    assert np.max(np.abs(inner(gT0) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC0) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


@pytest.mark.parametrize("periods", [(1, 1, 1), (1, 0, 1)])
def test_adjoint_seed_and_restriction(periods):
    """igg_adjoint_seed: lam = T - T_obs on the inner points with the halo of
    lam the periodic images (zero in non-periodic dimensions), the loss equal
    to igg_reduce(HALF_SQDIFF) bit for bit and to the exactly rounded sum;
    without T_obs it restricts T to the inner points, without T it zeroes."""
    n = (70, 36, 30)
    say("adjoint seed", periods)
    T0, Tobs = synth.uniform_fields(*n, seed=59, lo=0.3, hi=0.9, n=2)
    ref = np.zeros_like(T0)
    inner(ref)[...] = inner(T0) - inner(Tobs)
    oracle.halo(ref, (2, 2, 2), periods)
    L_exact = 0.5 * math.fsum((inner(T0) - inner(Tobs)).ravel() ** 2)
    with grid(n, periods):
        T, O = dev(T0), dev(Tobs)
        lam = torch.full_like(T, 7.0)
        L = igg.adjoint_seed(lam, T, O, halo=True, loss=True)
        assert L == igg.reduce(igg.RED_HALF_SQDIFF, T, O)
        assert abs(L - L_exact) <= 1e-13 * L_exact
        assert np.array_equal(host(lam), ref)
        r = torch.full_like(T, 7.0)
        assert igg.adjoint_seed(r, T, halo=False) is None
        want = np.zeros_like(T0)
        inner(want)[...] = inner(T0)
        assert np.array_equal(host(r), want)
        z = torch.full_like(T, 7.0)
        igg.adjoint_seed(z, halo=False)
        assert not torch.any(z != 0).item()
        with pytest.raises(igg.IggError):
            igg.adjoint_seed(lam, None, O)
        with pytest.raises(igg.IggError):
            igg.adjoint_seed(T, T, O)  # lam aliases T
