"""Parity at the benchmarked sizes, in the launch configuration bench.py
times (512^3, split (16,2,2), 100 steps): sampled outputs against the
oracle's light-cone evaluation, precision forms against their bounds, the
768^3 flux form, and remaining GPU cases (mixed periods, flux-form adjoint,
FP16 stochastic rounding)."""
import math

import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, inner, rel_max_err, say  # noqa: E402

SAMPLES = [(1, 1, 1), (510, 510, 510), (255, 256, 257), (100, 400, 17), (480, 3, 300), (16, 200, 509),
           (495, 2, 2), (17, 509, 128)]


def _oracle_samples(T0, Ci, nt, lam, dt, d, pts):
    return oracle.run_points(T0, Ci, nt, lam, dt, *d, pts)


def test_c2_512_fp64_samples_match_oracle():
    """512^3 FP64 bump + lognormal Ci, 100 boundary-first steps: eight
    sampled points (corners, slab edges, interior) against the oracle's
    light cone, <= 1e-12 relative."""
    say("c2 512^3 fp64")
    w = synth.workload("c2_512_fp64", seed=0)
    n = (w["nx"], w["ny"], w["nz"])
    nt, lam, d = w["nt"], w["lam"], (w["dx"], w["dy"], w["dz"])
    T0, Ci = w["T0"], w["Ci"]
    oracle.halo(T0)
    oracle.halo(Ci)
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    with grid(n):
        T, C = dev(T0), dev(Ci)
        assert igg.diffusion_dt(C, lam, *d) == dt
        out = diffusion.forward(T, C, nt, lam, dt, *d, split=(16, 2, 2))
        got = np.array([out[k, j, i].item() for (i, j, k) in SAMPLES])
        # the z halo planes of the result are the periodic images (full planes)
        assert torch.equal(out[0], out[-2]) and torch.equal(out[-1], out[1])
    ref = _oracle_samples(T0, Ci, nt, lam, dt, d, SAMPLES)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err


def test_c3_512_precision_forms_within_bounds():
    """512^3 noisy bump, uniform Ci, 100 steps: FP32 <= 1e-5 and FP16
    storage (stochastic rounding) <= 2e-3 relative max error against the FP64
    run over all unique points, and the FP64 run against the oracle on
    samples."""
    say("c3 512^3 precision")
    w = synth.workload("c3_512", seed=0)
    n = (w["nx"], w["ny"], w["nz"])
    nt, lam, d = w["nt"], w["lam"], (w["dx"], w["dy"], w["dz"])
    T0, Ci = w["T0"], w["Ci"]
    oracle.halo(T0)
    oracle.halo(Ci)
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    errs = {}
    with grid(n):
        T64, C64 = dev(T0), dev(Ci)
        ref = diffusion.forward(T64.clone(), C64, nt, lam, dt, *d)
        got64 = np.array([ref[k, j, i].item() for (i, j, k) in SAMPLES])
        rmax = ref[1:-1, 1:-1, 1:-1].abs().max().item()
        for name, tdt, seed in (("f32", torch.float32, None), ("f16", torch.float16, 11)):
            out = diffusion.forward(T64.to(tdt), C64.to(tdt), nt, lam, dt, *d, sr_seed=seed)
            errs[name] = (out.double() - ref)[1:-1, 1:-1, 1:-1].abs().max().item() / rmax
            del out
    say("errors", errs)
    assert errs["f32"] <= 1e-5
    assert errs["f16"] <= 2e-3
    ref_o = _oracle_samples(T0, Ci, nt, lam, dt, d, SAMPLES[:4])
    assert np.max(np.abs(got64[:4] - ref_o)) / np.max(np.abs(ref_o)) <= 1e-12


def test_c5_768_flux_form_fp32_vs_fp64():
    """768^3 staggered flux form, 100 steps with the four-field halo update
    every step: FP32 within 1e-5 of FP64, FP64 within 1e-12 of the Laplacian
    form on the same grid."""
    say("c5 768^3 flux")
    w = synth.workload("c5_768_flux", seed=0)
    n = (w["nx"], w["ny"], w["nz"])
    nz, ny, nx = w["T0"].shape
    nt, lam, d = w["nt"], w["lam"], (w["dx"], w["dy"], w["dz"])
    T0, Ci = w["T0"], w["Ci"]
    oracle.halo(T0)
    oracle.halo(Ci)
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    shapes = oracle.face_shapes(T0)
    outs = {}
    with grid(n):
        for name, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            T, C = dev(T0, tdt), dev(Ci, tdt)
            W = torch.empty_like(T)
            q = [torch.zeros(s, dtype=tdt, device="cuda") for s in shapes]
            for _ in range(nt):
                igg.diffusion_flux_step(W, T, C, *q, lam, dt, *d)
                T, W = W, T
            outs[name] = T.double()
            del W, q, C
            torch.cuda.empty_cache()
        lap = diffusion.forward(dev(T0), dev(Ci), nt, lam, dt, *d, split=None)
        rmax = outs["f64"][1:-1, 1:-1, 1:-1].abs().max().item()
        e32 = (outs["f32"] - outs["f64"])[1:-1, 1:-1, 1:-1].abs().max().item() / rmax
        e_lap = (lap - outs["f64"])[1:-1, 1:-1, 1:-1].abs().max().item() / rmax
    say("flux errors", e32, e_lap)
    assert e32 <= 1e-5
    assert e_lap <= 1e-12


@pytest.mark.parametrize("periods", [(1, 0, 1), (0, 1, 0), (0, 0, 0)])
def test_mixed_periods_match_oracle(periods):
    """Non-periodic dimensions keep their halo planes; periodic ones are
    updated.  Split and unsplit both match the oracle."""
    say("periods", periods)
    n = (70, 44, 38)
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=21, noise=1e-2)
    oracle.halo(T0, (2, 2, 2), periods)
    oracle.halo(Ci, (2, 2, 2), periods)
    d = (1 / 69, 1 / 43, 1 / 37)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, 9, 1.0, dt, *d, periods=periods)
    with grid(n, periods):
        for split in (None, (16, 2, 2)):
            out = diffusion.forward(dev(T0), dev(Ci), 9, 1.0, dt, *d, split=split)
            got = host(out)
            assert rel_max_err(got, ref) <= 1e-12
            # halo planes of non-periodic dimensions are untouched
            for dim, p in enumerate(periods):
                if not p:
                    sl = [slice(None)] * 3
                    sl[2 - dim] = 0
                    assert np.array_equal(got[tuple(sl)], T0[tuple(sl)])


def test_flux_adjoint_matches_oracle():
    say("flux adjoint")
    n = (34, 28, 24)
    nx, ny, nz = n
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=61, lo=0.3, hi=0.9, n=3)
    for a in (T0, Ci, Tobs):
        oracle.halo(a)
    d = (1 / 33, 1 / 27, 1 / 23)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 5
    L_ref, gT_ref, gC_ref = oracle.flux_gradient(T0, Ci, Tobs, nt, 1.0, dt, *d)
    shapes = oracle.face_shapes(T0)
    with grid(n):
        T, C, O = dev(T0), dev(Ci), dev(Tobs)
        states, fluxes = [T], []
        for _ in range(nt):
            W = torch.empty_like(T)
            q = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in shapes]
            igg.diffusion_flux_step(W, states[-1], C, *q, 1.0, dt, *d)
            states.append(W)
            fluxes.append(q)
        L = igg.reduce(igg.RED_HALF_SQDIFF, states[-1], O)
        lp = torch.zeros_like(T)
        lp[1:-1, 1:-1, 1:-1] = (states[-1] - O)[1:-1, 1:-1, 1:-1]
        igg.update_halo(lp)
        g = torch.zeros_like(T)
        for it in range(nt - 1, -1, -1):
            ln = torch.zeros_like(T)
            igg.diffusion_flux_step_adjoint(ln, lp, states[it], C, g, 1.0, dt, *d)
            lp = ln
        gT, gC = host(lp), host(g)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert np.max(np.abs(inner(gT) - inner(gT_ref))) <= 1e-12 * np.max(np.abs(inner(gT_ref)))
    assert np.max(np.abs(inner(gC) - inner(gC_ref))) <= 1e-12 * np.max(np.abs(inner(gC_ref)))


def test_fp16_stochastic_rounding_is_unbiased_and_deterministic():
    """A field whose exact update lands between FP16 values: one step with
    stochastic rounding gives values that average to the exact FP32 result
    (within a few standard errors), never leave the two neighbouring FP16
    values, repeat bit for bit with the same (seed, counter) and change with
    another counter."""
    say("fp16 SR")
    n = (256, 64, 32)
    nx, ny, nz = n
    x = synth.coords(nx)
    T0 = np.broadcast_to(1.7 + 0.05 * np.sin(2 * np.pi * x * 3), (nz, ny, nx)).copy()
    Ci = np.full((nz, ny, nx), 0.5)
    oracle.halo(T0)
    dx = 1 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, 0.5)
    with grid(n):
        T16 = dev(T0, torch.float16)
        C16 = dev(Ci, torch.float16)
        T32 = T16.float().contiguous()
        C32 = C16.float().contiguous()
        exact = torch.empty_like(T32)
        igg.diffusion_step(exact, T32, C32, 1.0, dt, dx, dx, dx, split=None)
        outs = []
        for c in range(3):
            o = torch.empty_like(T16)
            igg.diffusion_step(o, T16, C16, 1.0, dt, dx, dx, dx, split=None,
                               rnd=igg.rounding("stochastic", 99, c))
            outs.append(o)
        again = torch.empty_like(T16)
        igg.diffusion_step(again, T16, C16, 1.0, dt, dx, dx, dx, split=None, rnd=igg.rounding("stochastic", 99, 0))
        torch.cuda.synchronize()
        assert torch.equal(again, outs[0])
        assert not torch.equal(outs[0], outs[1])
        e = exact[1:-1, 1:-1, 1:-1].double()
        spacing = torch.pow(2.0, torch.floor(torch.log2(e.abs())) - 10)  # FP16 normal-range spacing
        for o in outs:
            v = o[1:-1, 1:-1, 1:-1].double()
            # one of the two FP16 values around the exact one
            assert torch.all(torch.abs(v - e) < spacing)
            assert torch.all(torch.floor(e / spacing) * spacing <= v)
            assert torch.all(v <= torch.ceil(e / spacing) * spacing)
        # unbiased: along each x line every point sees the same update, so the
        # mean over the (j, k) copies and the counters estimates the exact value
        m = torch.stack([o[1:-1, 1:-1, 1:-1].double() for o in outs]).mean(dim=(0, 1, 2))
        ex = e[0, 0]
        nsamp = 3 * (ny - 2) * (nz - 2)
        bound = 5 * spacing[0, 0] / math.sqrt(nsamp)
        assert torch.all(torch.abs(m - ex) <= bound)
        # round-to-nearest stores differ from the stochastic ones somewhere
        rn = torch.empty_like(T16)
        igg.diffusion_step(rn, T16, C16, 1.0, dt, dx, dx, dx, split=None)
        torch.cuda.synchronize()
        assert not torch.equal(rn, outs[0])


def _hashed_box(c, r, n, seed, offset):
    """Values of a periodic hashed field (overlap 2, halo = periodic images)
    on the padded index box c-r .. c+r around point c = (i, j, k)."""
    ax = [(np.arange(cd - r, cd + r + 1) - 1) % (nd - 2) + 1 for cd, nd in zip(c, n)]
    lin = ax[0][None, None, :] + n[0] * (ax[1][None, :, None] + n[1] * ax[2][:, None, None])
    return offset + synth.hashed_uniform(lin, seed)


def test_fp64_step_beyond_2_31_points_matches_oracle():
    """A grid of 1024 x 1024 x 2052 = 2.15e9 points (more than 2^31, so
    element indices need 64 bits; 17 GB per FP64 field), hashed uniform T in
    [1.5, 2.5) and Ci in [0.5, 1.5): two boundary-first steps, then sampled
    points -- among them points whose linear index exceeds 2^31 -- against
    the oracle's light cone, <= 1e-12 relative, and the halo planes of the
    result equal to their periodic images."""
    n = (1024, 1024, 2052)
    assert n[0] * n[1] * n[2] > 1 << 31
    lam, nt = 1.0, 2
    d = tuple(1.0 / (m - 1) for m in n)
    dt = oracle.time_step(*d, lam, 1.5)  # Ci < 1.5 everywhere
    pts = [(1, 1, 1), (1022, 1022, 2050), (700, 1000, 2049), (3, 2, 2050), (1022, 511, 2048), (512, 512, 1024),
           (16, 17, 2047), (1007, 1021, 2050)]
    assert max(i + n[0] * (j + n[1] * k) for i, j, k in pts) > 1 << 31
    say("fp64 beyond 2^31 points", n)
    with grid(n, zmarch_min=None):
        T = synth.hashed_field_torch(*n, 1, 1.5, "cuda")
        C = synth.hashed_field_torch(*n, 2, 0.5, "cuda")
        igg.update_halo(T, C)
        out = diffusion.forward(T, C, nt, lam, dt, *d, split=(16, 2, 2))
        got = np.array([out[k, j, i].item() for (i, j, k) in pts])
        assert torch.equal(out[0], out[-2]) and torch.equal(out[-1], out[1])
        assert torch.equal(out[:, 0], out[:, -2]) and torch.equal(out[:, -1], out[:, 1])
        assert torch.equal(out[:, :, 0], out[:, :, -2]) and torch.equal(out[:, :, -1], out[:, :, 1])
        del T, C, out
    ref = []
    for c in pts:
        Tb = _hashed_box(c, nt, n, 1, 1.5)
        Cb = _hashed_box(c, nt, n, 2, 0.5)
        ref.append(oracle.run(Tb, Cb, nt, lam, dt, *d, ol=(2, 2, 2), periods=(0, 0, 0))[nt, nt, nt])
    ref = np.array(ref)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err
