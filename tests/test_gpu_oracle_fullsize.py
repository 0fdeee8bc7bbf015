"""Full-field parity with the oracle at the benchmarked sizes, in the launch
configurations bench.py times: every unique point of the 512^3 FP64 run
(split (16, 2, 2), 100 steps, 16-plane z chunks), the FP32 and FP16-storage
forms against the FP64 oracle run, the 256^3 inverse-problem gradients
(nt = 200, snapshots every 16) against the oracle's adjoint sweep, and the
staggered flux form against the oracle's flux loop on a multi-tile grid and
at 768^3 on light-cone samples, and one adjoint step (both forms) on a region
above 2^26 points, where the adjoint kernel takes its 1024-thread tiles.

The inputs are the seeded workload recipes; every expected value comes from
the oracle."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, inner, rel_max_err, say  # noqa: E402


def _prepared(name):
    w = synth.workload(name, seed=0)
    T0, Ci = w["T0"], w["Ci"]
    oracle.halo(T0)
    oracle.halo(Ci)
    n = (w["nx"], w["ny"], w["nz"])
    d = (w["dx"], w["dy"], w["dz"])
    return w, T0, Ci, n, d


def _halo_is_periodic_image(t):
    """Every halo plane of a periodic overlap-2 field equals its image."""
    return (torch.equal(t[0], t[-2]) and torch.equal(t[-1], t[1]) and torch.equal(t[:, 0], t[:, -2])
            and torch.equal(t[:, -1], t[:, 1]) and torch.equal(t[:, :, 0], t[:, :, -2])
            and torch.equal(t[:, :, -1], t[:, :, 1]))


def test_c2_512_fp64_full_field_matches_oracle():
    """512^3 bump + lognormal Ci, 100 boundary-first steps (16, 2, 2): every
    unique point within 1e-12 of the oracle, halo planes the exact periodic
    images, and the GPU's dt equal to the oracle's bit for bit."""
    say("c2 512^3 fp64 full field")
    w, T0, Ci, n, d = _prepared("c2_512_fp64")
    nt, lam = w["nt"], w["lam"]
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    with grid(n, zmarch_min=None):
        T, C = dev(T0), dev(Ci)
        assert igg.diffusion_dt(C, lam, *d) == dt
        out = diffusion.forward(T, C, nt, lam, dt, *d, split=(16, 2, 2))
        assert _halo_is_periodic_image(out)
        got = host(out)
        del T, C, out
    ref = oracle.run(T0, Ci, nt, lam, dt, *d)
    err = rel_max_err(got, ref)
    say("c2 error", err)
    assert err <= 1e-12, err


def test_c3_512_precision_forms_match_fp64_oracle():
    """512^3 noisy bump, uniform Ci, 100 boundary-first steps: FP64 within
    1e-12, FP32 within 1e-5 and FP16 storage with stochastic rounding within
    2e-3 of the FP64 oracle run, over every unique point."""
    say("c3 512^3 precision forms vs oracle")
    w, T0, Ci, n, d = _prepared("c3_512")
    nt, lam = w["nt"], w["lam"]
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    ref = oracle.run(T0, Ci, nt, lam, dt, *d)
    errs = {}
    with grid(n, zmarch_min=None):
        for name, tdt, seed in (("f64", torch.float64, None), ("f32", torch.float32, None),
                                ("f16", torch.float16, 11)):
            say("c3", name)
            T, C = diffusion.prepare_fields(T0, Ci, tdt)
            out = diffusion.forward(T, C, nt, lam, dt, *d, split=(16, 2, 2), sr_seed=seed)
            errs[name] = rel_max_err(host(out), ref)
            del T, C, out
            torch.cuda.empty_cache()
    say("c3 errors", errs)
    assert errs["f64"] <= 1e-12
    assert errs["f32"] <= 1e-5
    assert errs["f16"] <= 2e-3


def test_c4_256_inverse_gradients_match_oracle():
    """256^3 FP64 inverse problem, nt = 200: T_obs is the oracle's forward
    run with the sine Ci_true, the guess is Ci = 0.5, dt is fixed from
    max(Ci_true).  The GPU's loss and both gradients (snapshots every 16,
    boundary-first adjoint steps) match the oracle's adjoint sweep with the
    same snapshots within 1e-12."""
    say("c4 256^3 gradients vs oracle")
    w, T0, Ctrue, n, d = _prepared("c4_256_inverse")
    nt, lam = w["nt"], w["lam"]
    dt = oracle.time_step(*d, lam, oracle.max_all(Ctrue))
    Tobs = oracle.run(T0, Ctrue, nt, lam, dt, *d)
    Cg = np.full_like(T0, 0.5)
    L_ref, gT_ref, gC_ref = oracle.gradient(T0, Cg, Tobs, nt, lam, dt, *d, every=16)
    with grid(n, zmarch_min=None):
        prob = diffusion.Problem(lam, dt, *d, split=(16, 2, 2))
        L, gT, gC, sw = diffusion.loss_and_grad(dev(T0), dev(Cg), dev(Tobs), prob, nt, ("periodic", 16))
        assert sw.adjoints == nt
        gT, gC = host(gT), host(gC)
    eL = abs(L - L_ref) / L_ref
    eT = np.max(np.abs(inner(gT) - inner(gT_ref))) / np.max(np.abs(inner(gT_ref)))
    eC = np.max(np.abs(inner(gC) - inner(gC_ref))) / np.max(np.abs(inner(gC_ref)))
    say("c4 errors", eL, eT, eC)
    assert eL <= 1e-12 and eT <= 1e-12 and eC <= 1e-12


@pytest.mark.parametrize("split", [None, (16, 3, 3)])
def test_flux_form_multi_tile_matches_oracle(split):
    """The fused flux pass on a grid spanning several x tiles of both
    precisions (256 FP32 cells, 128 FP64 cells per tile row), several tile
    rows and z chunks, with ragged tails: T2 and the three face fields
    within 1e-12 (FP64) and T2 within 1e-5 (FP32) of the oracle's flux
    loop after 12 steps."""
    say("flux multi-tile vs oracle", split)
    n = (530, 46, 41)
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=71, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    d = (1 / 529, 1 / 45, 1 / 40)
    lam, nt = 1.0, 12
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    ref, qref = oracle.flux_run(T0, Ci, nt, lam, dt, *d, return_q=True)
    with grid(n):
        for tdt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
            prob = diffusion.FluxProblem(lam, dt, *d, split=split)
            T, C = dev(T0, tdt), dev(Ci, tdt)
            out = diffusion.forward_with(prob, T, C, nt)
            err = rel_max_err(host(out), ref)
            say("flux", tdt, err)
            assert err <= tol, (tdt, err)
            if tdt == torch.float64:
                for q, qr in zip(prob.fluxes, qref):
                    qh = host(q)
                    eq = np.max(np.abs(qh - qr)) / np.max(np.abs(qr))
                    assert eq <= 1e-12, eq


def test_c5_768_flux_form_samples_match_oracle():
    """768^3 staggered flux form, 100 steps in FP64 and FP32: three sampled
    cells (a corner, a tile edge, the interior) against the oracle's
    flux-form light cone, FP64 within 1e-12 and FP32 within 1e-5."""
    say("c5 768^3 flux samples vs oracle")
    w, T0, Ci, n, d = _prepared("c5_768_flux")
    nt, lam = w["nt"], w["lam"]
    dt = oracle.time_step(*d, lam, oracle.max_all(Ci))
    pts = [(1, 1, 1), (256, 383, 700), (766, 2, 384)]
    got = {}
    with grid(n, zmarch_min=None):
        for name, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            say("c5", name)
            prob = diffusion.FluxProblem(lam, dt, *d)
            T, C = diffusion.prepare_fields(T0, Ci, tdt)
            out = diffusion.forward_with(prob, T, C, nt)
            got[name] = np.array([out[k, j, i].item() for (i, j, k) in pts])
            del T, C, out, prob
            torch.cuda.empty_cache()
    ref = oracle.flux_run_points(T0, Ci, nt, lam, dt, *d, pts)
    e64 = np.max(np.abs(got["f64"] - ref)) / np.max(np.abs(ref))
    e32 = np.max(np.abs(got["f32"] - ref)) / np.max(np.abs(ref))
    say("c5 errors", e64, e32)
    assert e64 <= 1e-12 and e32 <= 1e-5


@pytest.mark.parametrize("form", ["laplacian", "flux"])
def test_adjoint_step_large_region_matches_oracle(form):
    """One adjoint step on a region of more than 2^26 points (the FP64
    kernel's 16-row tiles of 1024 threads, as at 512^3) against the oracle's
    adjoint step at every inner point: lam_n and the accumulated gCi, for the
    Laplacian form and the flux form (whose fluxes the oracle forms from T_n
    with its own flux routine)."""
    n = (424, 420, 416)
    nx, ny, nz = n
    assert (nx - 2) * (ny - 2) * (nz - 2) >= 2 ** 26
    say("adjoint large region", form)
    rng = np.random.default_rng(23)
    lp = rng.uniform(-1.0, 1.0, (nz, ny, nx))
    Tn = rng.uniform(1.0, 2.0, (nz, ny, nx))
    Ci = rng.uniform(0.5, 1.5, (nz, ny, nx))
    g0 = rng.uniform(-1.0, 1.0, (nz, ny, nx))
    for a in (lp, Tn, Ci):
        oracle.halo(a)
    dx, dy, dz = 1 / (nx - 1), 1 / (ny - 1), 1 / (nz - 1)
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    g_ref = g0.copy()
    if form == "laplacian":
        ln_ref = oracle.adjoint_step(lp, Tn, Ci, g_ref, 1.0, dt, dx, dy, dz)
    else:
        q = oracle.flux(Tn, 1.0, dx, dy, dz)
        ln_ref = oracle.flux_adjoint_step(lp, Ci, q, g_ref, 1.0, dt, dx, dy, dz)
        del q
    with grid(n):
        lpd, Tnd, Cid, gd = dev(lp), dev(Tn), dev(Ci), dev(g0)
        lnd = torch.zeros_like(lpd)
        if form == "laplacian":
            igg.diffusion_step_adjoint(lnd, lpd, Tnd, Cid, gd, 1.0, dt, dx, dy, dz, split=None)
        else:
            igg.diffusion_flux_step_adjoint(lnd, lpd, Tnd, Cid, gd, 1.0, dt, dx, dy, dz, split=None)
        ln, g = host(lnd), host(gd)
    assert rel_max_err(ln, ln_ref) <= 1e-12
    assert rel_max_err(g, g_ref) <= 1e-12
