"""Parity of the HIP path (through the C ABI) with the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_common import PER, dev, grid, host, inner, rel_max_err, say  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def _image(n, ol):
    img = np.arange(n)
    img[0] = n - ol
    img[n - 1] = ol - 1
    return img


# --------------------------------------------------------------------------- halo
@pytest.mark.parametrize("n,periods", [((3, 3, 3), PER), ((4, 5, 6), PER), ((7, 3, 5), (1, 0, 1)),
                                       ((33, 17, 9), PER), ((40, 34, 21), (0, 1, 1))])
@pytest.mark.parametrize("dt", ["f64", "f32", "f16"])
def test_halo_bit_exact(n, periods, dt):
    say("halo", n, periods, dt)
    nx, ny, nz = n
    rng = np.random.default_rng(21)
    shapes = [(nz, ny, nx), (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
    arrs = [rng.uniform(-1, 1, s) for s in shapes]
    with grid(n, periods):
        ts = [dev(a, DT[dt]) for a in arrs]
        igg.update_halo(*ts)
        for a, t in zip(arrs, ts):
            ref = host(dev(a, DT[dt]))  # the same rounding of the input
            sz, sy, sx = a.shape
            ol = [2 + (s - m) for s, m in zip((sx, sy, sz), n)]
            imgs = [(_image(s, o) if p else np.arange(s)) for s, o, p in zip((sx, sy, sz), ol, periods)]
            expect = ref[np.ix_(imgs[2], imgs[1], imgs[0])]
            assert np.array_equal(host(t), expect)


def test_halo_matches_oracle_mixed_fields():
    say("halo mixed dtypes vs oracle")
    n = (20, 18, 16)
    rng = np.random.default_rng(3)
    a = rng.uniform(0, 1, (16, 18, 21))
    b = rng.uniform(0, 1, (16, 18, 20))
    with grid(n):
        ta, tb = dev(a), dev(b, torch.float32)
        igg.update_halo(ta, tb)
        ea = oracle.halo(a.copy(), (3, 2, 2), PER)
        eb = oracle.halo(host(dev(b, torch.float32)), (2, 2, 2), PER)
        assert np.array_equal(host(ta), ea)
        assert np.array_equal(host(tb), eb)


# --------------------------------------------------------------------------- forward FP64
def _setup(name, n=None, seed=0):
    w = synth.workload(name, seed=seed, n=n)
    T0, Ci = w["T0"].copy(), w["Ci"].copy()
    oracle.halo(T0)
    oracle.halo(Ci)
    return w, T0, Ci


@pytest.mark.parametrize("split", [(16, 2, 2), None, (2, 2, 2), (5, 3, 4)])
def test_c1_forward_matches_oracle(split):
    """32^3 FP64, nt=10, periodic, halo every step: <= 1e-12 relative."""
    say("c1 forward", split)
    w, T0, Ci = _setup("c1_32_fp64")
    n = (w["nx"], w["ny"], w["nz"])
    dx, dy, dz, lam, nt = w["dx"], w["dy"], w["dz"], w["lam"], w["nt"]
    dt_o = oracle.time_step(dx, dy, dz, lam, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, nt, lam, dt_o, dx, dy, dz)
    with grid(n):
        T, C = diffusion.prepare_fields(w["T0"], w["Ci"])
        assert np.array_equal(host(T), T0) and np.array_equal(host(C), Ci)
        dt = igg.diffusion_dt(C, lam, dx, dy, dz)
        assert dt == dt_o
        out = diffusion.forward(T, C, nt, lam, dt, dx, dy, dz, split=split)
        got = host(out)
    assert rel_max_err(got, ref) <= 1e-12
    # the halo of the result is the periodic image of its inner points
    assert np.array_equal(got, oracle.halo(got.copy()))


@pytest.mark.parametrize("n", [(67, 45, 38), (130, 70, 40), (33, 9, 11), (64, 64, 64)])
@pytest.mark.parametrize("mid", [None, "0"])
def test_forward_ragged_sizes(n, mid, monkeypatch):
    """Sizes spanning several tiles with ragged tails, odd nx (scalar path);
    FP64 tiles of both shapes (mid = "0" forces the large-region one)."""
    if mid is not None:
        monkeypatch.setenv("IGG_FP64_MIDTILE_MAX_POINTS", mid)
    say("forward ragged", n, mid)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=5, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx, dy, dz = 1 / (nx - 1), 1 / (ny - 1), 1 / (nz - 1)
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, 7, 1.0, dt, dx, dy, dz)
    with grid(n):
        T, C = dev(T0), dev(Ci)
        for split in [(16, 2, 2), None]:
            out = diffusion.forward(T.clone(), C, 7, 1.0, dt, dx, dy, dz, split=split)
            assert rel_max_err(host(out), ref) <= 1e-12


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_split_equals_unsplit_bit_exact(dt_name):
    say("split vs unsplit", dt_name)
    n = (96, 52, 41)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=9, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    with grid(n):
        T, C = dev(T0, DT[dt_name]), dev(Ci, DT[dt_name])
        outs = []
        for split in [None, (16, 2, 2), (2, 2, 2), (17, 5, 3), (60, 30, 30)]:
            o = diffusion.forward(T.clone(), C, 6, 1.0, dt, dx, dx, dx, split=split,
                                  sr_seed=7 if dt_name == "f16" else None)
            outs.append(host(o))
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("n", [(260, 40, 20), (300, 35, 19), (60, 30, 20), (131, 22, 18)])
@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
@pytest.mark.parametrize("xform", ["fused", "halo"])
def test_wide_rows_split_forms(n, dt_name, xform, monkeypatch):
    """With the x exchange as a separate pass of the halo update the x slabs
    are computed first: slabs up to 31 points wide take the 64-point wrapped
    tiles, 32 to 64 points the 128-point wrapped tiles with their outer x
    neighbours, rows below 64 points (or odd) the narrow tiles.  With the
    fused exchange they join the inner launch.  Every result equals the
    unsplit step, and FP64 the oracle."""
    monkeypatch.setenv("IGG_X_EXCHANGE", xform)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=19, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, 4, 1.0, dt, dx, dx, dx) if dt_name == "f64" else None
    outs = []
    with grid(n):
        T, C = dev(T0, DT[dt_name]), dev(Ci, DT[dt_name])
        for split in [None, (16, 2, 2), (64, 2, 2), (40, 2, 2), (63, 2, 3), (31, 2, 2), (32, 2, 2), (2, 5, 3)]:
            say("wide rows", n, dt_name, split)
            o = diffusion.forward(T.clone(), C, 4, 1.0, dt, dx, dx, dx, split=split,
                                  sr_seed=7 if dt_name == "f16" else None)
            outs.append(host(o))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    if ref is not None:
        assert rel_max_err(outs[0], ref) <= 1e-12


@pytest.mark.parametrize("n,ol,periods,splits", [
    ((70, 30, 26), (3, 2, 2), (1, 1, 1), [None, (16, 4, 4), (3, 2, 2)]),
    ((70, 30, 26), (4, 3, 2), (1, 0, 1), [None, (16, 4, 4), (5, 3, 2)]),
    ((140, 24, 20), (3, 2, 3), (1, 1, 1), [None, (40, 3, 3), (64, 2, 3), (16, 2, 3)]),
    ((66, 20, 18), (2, 2, 2), (0, 1, 1), [None, (16, 2, 2)]),
])
def test_wider_overlaps_match_oracle(n, ol, periods, splits):
    """Overlaps above 2: the x halo of the result is the column ol-1 / nx-ol
    copy, stored by the kernels that compute those columns, for every split
    form (narrow, 64- and 128-point wrapped x slabs) and the unsplit step."""
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=23, noise=1e-2)
    oracle.halo(T0, ol, periods)
    oracle.halo(Ci, ol, periods)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, 5, 1.0, dt, dx, dx, dx, ol=ol, periods=periods)
    with grid(n, periods, ol):
        T, C = dev(T0), dev(Ci)
        for split in splits:
            say("wider overlaps", n, ol, periods, split)
            got = host(diffusion.forward(T.clone(), C, 5, 1.0, dt, dx, dx, dx, split=split))
            # every point, halos included: the non-periodic halo planes keep T0's values
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
            assert np.array_equal(got, oracle.halo(got.copy(), ol, periods))


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_schedules_and_x_exchange_forms_bit_exact(dt_name, monkeypatch):
    """Every schedule (slabs and update on the helper stream beside the inner
    region, slabs on the caller stream before it, or one chain on the caller
    stream) and both x-exchange forms (fused into the
    step kernels' stores with the x slabs in the inner launch, or a separate
    x pass of the halo update with the x slabs in the boundary phase) give
    the same bits, halos included, as the unsplit step."""
    n = (96, 52, 41)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=29, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    outs = []
    for sched in ("1", "0", "2", "3"):
        for xform in ("fused", "halo"):
            monkeypatch.setenv("IGG_SCHEDULE", sched)
            monkeypatch.setenv("IGG_X_EXCHANGE", xform)
            with grid(n):
                T, C = dev(T0, DT[dt_name]), dev(Ci, DT[dt_name])
                for split in [None, (16, 2, 2), (3, 4, 2)]:
                    say("schedule", sched, "x exchange", xform, dt_name, split)
                    o = diffusion.forward(T.clone(), C, 5, 1.0, dt, dx, dx, dx, split=split,
                                          sr_seed=7 if dt_name == "f16" else None)
                    outs.append(host(o))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("n", [(32, 32, 32), (96, 52, 41), (130, 70, 40), (33, 9, 11)])
@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_box_kernel_and_zmarch_paths_bit_exact(n, dt_name, monkeypatch):
    """Small regions go to the one-thread-per-point box kernel by default;
    forced through the z-march kernels (FP64: both tile shapes, the 512-thread
    one of mid-sized regions and the 256-thread one of large regions) they
    give the same bits."""
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=31, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    outs = []
    for zmin, mid in ((None, None), (0, None), (0, "0")):
        if mid is None:
            monkeypatch.delenv("IGG_FP64_MIDTILE_MAX_POINTS", raising=False)
        else:
            monkeypatch.setenv("IGG_FP64_MIDTILE_MAX_POINTS", mid)
        with grid(n, zmarch_min=zmin):
            T, C = dev(T0, DT[dt_name]), dev(Ci, DT[dt_name])
            for split in [None, (16, 2, 2)]:
                say("box vs zmarch", n, dt_name, zmin, split)
                o = diffusion.forward(T.clone(), C, 4, 1.0, dt, dx, dx, dx, split=split,
                                      sr_seed=7 if dt_name == "f16" else None)
                outs.append(host(o))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_constant_state_exact_all_dtypes(dt_name):
    """Fig. 1's own state (T = 1.7, Ci = 1/c0) never changes, in any precision."""
    say("constant state", dt_name)
    n = (48, 40, 36)
    with grid(n):
        T = torch.full((36, 40, 48), 1.7, dtype=DT[dt_name], device="cuda")
        C = torch.full_like(T, 0.5)
        ref = T.clone()
        dx = 1.0 / 47
        dt = igg.diffusion_dt(C, 1.0, dx, dx, dx)
        out = diffusion.forward(T, C, 25, 1.0, dt, dx, dx, dx, sr_seed=3 if dt_name == "f16" else None)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_fourier_mode_closed_form_on_gpu():
    say("fourier")
    nx, ny, nz = 34, 26, 30
    m = (2, 1, 3)
    dx, dy, dz = 1 / 33, 1.2 / 25, 0.9 / 29
    T0 = synth.fourier_mode(nx, ny, nz, m, 1.7, 0.1)
    c, nt = 0.5, 20
    dt = oracle.time_step(dx, dy, dz, 1.0, c)
    G = 1 - dt * c * sum(4 / d**2 * math.sin(math.pi * md / (n - 2)) ** 2
                         for md, n, d in zip(m, (nx, ny, nz), (dx, dy, dz)))
    expect = 1.7 + 0.1 * G**nt * (T0 - 1.7) / 0.1
    with grid((nx, ny, nz)):
        T, C = dev(T0), torch.full((nz, ny, nx), c, dtype=torch.float64, device="cuda")
        out = host(diffusion.forward(T, C, nt, 1.0, dt, dx, dy, dz))
    assert np.max(np.abs(out - expect)) <= 1e-12 * 0.1


def test_reductions_match_exact_sums():
    say("reductions")
    n = (40, 33, 29)
    a, b = synth.uniform_fields(*n, seed=17, lo=0.5, hi=1.5, n=2)
    with grid(n):
        ta, tb = dev(a), dev(b)
        ia, ib = inner(a).ravel(), inner(b).ravel()
        assert igg.reduce(igg.RED_MAX, ta) == a.max()
        assert igg.reduce(igg.RED_MIN, ta) == a.min()
        assert igg.reduce(igg.RED_MAX_ABS_DIFF, ta, tb) == np.max(np.abs(ia - ib))
        for op, exact in [(igg.RED_SUM, math.fsum(ia)), (igg.RED_SUM_RATIO, math.fsum(ia / ib)),
                          (igg.RED_DOT, math.fsum(ia * ib)),
                          (igg.RED_HALF_SQDIFF, 0.5 * math.fsum((ia - ib) ** 2))]:
            got = igg.reduce(op, ta, tb)
            assert abs(got - exact) <= 1e-13 * abs(exact)
            assert igg.reduce(op, ta, tb) == got  # deterministic
        # FP32 / FP16 inputs are widened to FP64 before summing
        t32 = dev(a, torch.float32)
        exact32 = math.fsum(inner(host(t32)).ravel())
        assert abs(igg.reduce(igg.RED_SUM, t32) - exact32) <= 1e-13 * exact32


def test_conservation_on_gpu():
    say("conservation")
    n = (60, 50, 40)
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=2, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1 / 59
    with grid(n):
        T, C = dev(T0), dev(Ci)
        dt = igg.diffusion_dt(C, 1.0, dx, dx, dx)
        s0 = igg.reduce(igg.RED_SUM_RATIO, T, C)
        out = diffusion.forward(T, C, 30, 1.0, dt, dx, dx, dx)
        s1 = igg.reduce(igg.RED_SUM_RATIO, out, C)
    assert abs(s1 - s0) <= 1e-12 * abs(s0)


# --------------------------------------------------------------------------- adjoint
def _adjoint_gpu(T0, Ci, Tobs, nt, lam, dt, dx, dy, dz, split):
    """Store-all forward + reverse sweep through the C ABI."""
    T, C, O = dev(T0), dev(Ci), dev(Tobs)
    states = [T]
    for _ in range(nt):
        nxt = torch.empty_like(T)
        igg.diffusion_step(nxt, states[-1], C, lam, dt, dx, dy, dz, split=split)
        states.append(nxt)
    lp = torch.zeros_like(T)
    lp[1:-1, 1:-1, 1:-1] = states[-1][1:-1, 1:-1, 1:-1] - O[1:-1, 1:-1, 1:-1]
    igg.update_halo(lp)
    g = torch.zeros_like(T)
    for it in range(nt - 1, -1, -1):
        ln = torch.zeros_like(T)
        igg.diffusion_step_adjoint(ln, lp, states[it], C, g, lam, dt, dx, dy, dz, split=split)
        lp = ln
    return host(lp), host(g)


@pytest.mark.parametrize("split", [None, (16, 2, 2), (3, 4, 2)])
def test_adjoint_matches_oracle(split):
    say("adjoint", split)
    n = (44, 30, 26)
    nx, ny, nz = n
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=31, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a)
    dx, dy, dz = 1 / 43, 1 / 29, 1 / 25
    nt = 8
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    _, gT_ref, gC_ref = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    with grid(n):
        gT, gC = _adjoint_gpu(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz, split)
    assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


# --------------------------------------------------------------------------- flux form
def test_flux_form_matches_oracle():
    say("flux form")
    n = (36, 28, 22)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=4, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx, dy, dz = 1 / 35, 1 / 27, 1 / 21
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    nt = 6
    ref, qref = oracle.flux_run(T0, Ci, nt, 1.0, dt, dx, dy, dz, return_q=True)
    with grid(n):
        T, C = dev(T0), dev(Ci)
        T2 = torch.empty_like(T)
        q = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in oracle.face_shapes(T0)]
        for _ in range(nt):
            igg.diffusion_flux_step(T2, T, C, *q, 1.0, dt, dx, dy, dz)
            T, T2 = T2, T
        got = host(T)
        qs = [host(x) for x in q]
    assert rel_max_err(got, ref) <= 1e-12
    for a, b in zip(qs, qref):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("periods", [(1, 1, 1), (0, 1, 1), (1, 0, 1)])
def test_flux_form_splits_schedules_and_x_forms(periods, monkeypatch):
    """The fused flux-form step under every split (widths >= overlap + 1),
    schedule and x-exchange form: T and the three face fields equal the
    unsplit run bit for bit, halos included, and the oracle within 1e-12."""
    n = (70, 30, 26)
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=8, noise=1e-2)
    oracle.halo(T0, (2, 2, 2), periods)
    oracle.halo(Ci, (2, 2, 2), periods)
    d = (1 / 69, 1 / 29, 1 / 25)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 5
    ref, qref = oracle.flux_run(T0, Ci, nt, 1.0, dt, *d, periods=periods, return_q=True)
    outs = []
    for sched, xform in (("1", "fused"), ("0", "halo"), ("2", "fused"), ("1", "halo")):
        monkeypatch.setenv("IGG_SCHEDULE", sched)
        monkeypatch.setenv("IGG_X_EXCHANGE", xform)
        with grid(n, periods):
            for split in [None, (16, 3, 3), (3, 3, 3), (5, 4, 3)]:
                say("flux", periods, sched, xform, split)
                T, C = dev(T0), dev(Ci)
                T2 = T.clone()
                q = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in oracle.face_shapes(T0)]
                for _ in range(nt):
                    igg.diffusion_flux_step(T2, T, C, *q, 1.0, dt, *d, split=split)
                    T, T2 = T2, T
                outs.append([host(T)] + [host(x) for x in q])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    assert np.max(np.abs(outs[0][0] - ref)) <= 1e-12 * np.max(np.abs(ref))
    for a, b in zip(outs[0][1:], qref):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_flux_split_below_face_overlap_is_rejected():
    with grid((20, 18, 16)):
        T = torch.ones((16, 18, 20), dtype=torch.float64, device="cuda")
        q = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in oracle.face_shapes(host(T))]
        with pytest.raises(igg.IggError):
            igg.diffusion_flux_step(T.clone(), T, T, *q, 1.0, 1e-4, 0.1, 0.1, 0.1, split=(16, 2, 2))
