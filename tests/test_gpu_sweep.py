"""Randomised parity sweep and extreme shapes: grid sizes from the smallest
allowed (n = ol + 1) up, random periods, overlaps 2-4, split widths from the
overlap up, every dtype; and long thin grids whose index products are large."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, say  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def _cases(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ol = tuple(int(v) for v in rng.integers(2, 5, size=3))
        n = tuple(int(rng.integers(o + 1, o + 1 + int(rng.choice([2, 9, 40, 90])))) for o in ol)
        periods = tuple(int(v) for v in rng.integers(0, 2, size=3))
        split = None if rng.random() < 0.3 else tuple(int(rng.integers(o, o + 20)) for o in ol)
        out.append((n, ol, periods, split))
    return out


@pytest.mark.parametrize("case", _cases(24, 2024))
@pytest.mark.parametrize("zmin", [0, None])
def test_random_grids_match_oracle(case, zmin):
    """FP64 against the oracle (all points, halos included); FP32 and FP16
    (stochastic rounding) split against unsplit bit for bit."""
    n, ol, periods, split = case
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=sum(n), noise=1e-2)
    oracle.halo(T0, ol, periods)
    oracle.halo(Ci, ol, periods)
    d = tuple(1.0 / (m - 1) for m in n)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 3
    ref = oracle.run(T0, Ci, nt, 1.0, dt, *d, ol=ol, periods=periods)
    with grid(n, periods, ol, zmarch_min=zmin):
        say("random grid", n, ol, periods, split, zmin)
        got = host(diffusion.forward(dev(T0), dev(Ci), nt, 1.0, dt, *d, split=split))
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        for name in ("f32", "f16"):
            seed = 3 if name == "f16" else None
            a = host(diffusion.forward(dev(T0, DT[name]), dev(Ci, DT[name]), nt, 1.0, dt, *d, split=split,
                                       sr_seed=seed))
            b = host(diffusion.forward(dev(T0, DT[name]), dev(Ci, DT[name]), nt, 1.0, dt, *d, split=None,
                                       sr_seed=seed))
            assert np.array_equal(a, b), name


def _adjoint_cases(count, seed):
    """Every other case periodic in all dimensions (one rank: the adjoint
    kernel stores the y/z halo of lambda from their images)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        ol = tuple(int(v) for v in rng.integers(2, 5, size=3))
        n = tuple(int(rng.integers(o + 1, o + 1 + int(rng.choice([2, 9, 40, 90])))) for o in ol)
        periods = (1, 1, 1) if q % 2 == 0 else tuple(int(v) for v in rng.integers(0, 2, size=3))
        split = None if rng.random() < 0.25 else tuple(int(rng.integers(o, o + 20)) for o in ol)
        out.append((n, ol, periods, split))
    return out


@pytest.mark.parametrize("case", _adjoint_cases(16, 77))
@pytest.mark.parametrize("zmin", [0, None])
@pytest.mark.parametrize("form", ["laplacian", "flux"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_grids_adjoint_step_matches_oracle(case, zmin, form, dtype):
    """One adjoint step, Laplacian and staggered flux form, against the
    oracle's adjoint step and halo update: lambda_n at every point (halos
    included: periodic images, zero in non-periodic dimensions) and the Ci
    gradient on the inner points; FP64 within 1e-12, FP32 (inputs rounded to
    FP32 for both sides) within 1e-5.  The flux form's split widths are at
    least ol+1."""
    n, ol, periods, split = case
    if form == "flux" and split is not None:
        split = tuple(max(w, o + 1) for w, o in zip(split, ol))
    nx, ny, nz = n
    lp, Tn, Ci, g0 = synth.uniform_fields(nx, ny, nz, seed=sum(n) + 1, lo=0.2, hi=1.0, n=4)
    if dtype == "f32":
        lp, Tn, Ci, g0 = (a.astype(np.float32).astype(np.float64) for a in (lp, Tn, Ci, g0))
    for a in (lp, Tn, Ci):
        oracle.halo(a, ol, periods)
    d = tuple(1.0 / (m - 1) for m in n)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    g_ref = g0.copy()
    if form == "flux":
        ref = oracle.flux_adjoint_step(lp, Ci, oracle.flux(Tn, 1.0, *d), g_ref, 1.0, dt, *d)
    else:
        ref = oracle.adjoint_step(lp, Tn, Ci, g_ref, 1.0, dt, *d)
    oracle.halo(ref, ol, periods)
    with grid(n, periods, ol, zmarch_min=zmin):
        say("random grid adjoint", form, dtype, n, ol, periods, split, zmin)
        t = DT[dtype]
        ln = torch.zeros(lp.shape, dtype=t, device="cuda")
        gC = dev(g0, t)
        step = igg.diffusion_flux_step_adjoint if form == "flux" else igg.diffusion_step_adjoint
        step(ln, dev(lp, t), dev(Tn, t), dev(Ci, t), gC, 1.0, dt, *d, split=split)
        got, g = host(ln).astype(np.float64), host(gC).astype(np.float64)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
    i3 = (slice(1, -1),) * 3
    assert np.max(np.abs(g[i3] - g_ref[i3])) <= tol * np.max(np.abs(g_ref[i3]))


@pytest.mark.parametrize("case", _adjoint_cases(16, 91))
@pytest.mark.parametrize("zmin", [0, None])
def test_random_grids_flux_form_matches_oracle(case, zmin):
    """Three FP64 steps of the staggered flux form against the oracle: the
    cell field and the three face fields at every point (halos included);
    split widths at least ol+1."""
    n, ol, periods, split = case
    if split is not None:
        split = tuple(max(w, o + 1) for w, o in zip(split, ol))
    nx, ny, nz = n
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=sum(n) + 2, noise=1e-2)
    oracle.halo(T0, ol, periods)
    oracle.halo(Ci, ol, periods)
    d = tuple(1.0 / (m - 1) for m in n)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 3
    ref, qref = oracle.flux_run(T0, Ci, nt, 1.0, dt, *d, overlaps=ol, periods=periods, return_q=True)
    with grid(n, periods, ol, zmarch_min=zmin):
        say("random grid flux", n, ol, periods, split, zmin)
        T, C = dev(T0), dev(Ci)
        T2 = T.clone()
        q = [torch.zeros(sh, dtype=torch.float64, device="cuda") for sh in oracle.face_shapes(T0)]
        for _ in range(nt):
            igg.diffusion_flux_step(T2, T, C, *q, 1.0, dt, *d, split=split)
            T, T2 = T2, T
        got = [host(T)] + [host(x) for x in q]
    assert np.max(np.abs(got[0] - ref)) <= 1e-12 * np.max(np.abs(ref))
    for a, b in zip(got[1:], qref):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("n,split", [((4096, 4096, 6), (16, 2, 2)), ((6, 6, 1 << 22), None)])
def test_extreme_aspect_ratios(n, split):
    """Grids of 10^8 points in a long thin shape (a 16.8 M-point plane, a
    4 M-plane column): sampled points against the oracle's light cone after
    3 steps, and the periodic halo of the result."""
    nx, ny, nz = n
    rng = np.random.default_rng(9)
    T0 = 1.7 + 1e-2 * rng.standard_normal((nz, ny, nx))
    Ci = rng.uniform(0.25, 0.75, (nz, ny, nx))
    oracle.halo(T0)
    oracle.halo(Ci)
    d = (1.0 / (nx - 1), 1.0 / (ny - 1), 1.0 / (nz - 1))
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 3
    pts = [(1, 1, 1), (nx - 2, ny - 2, nz - 2), (nx // 2, ny // 3, nz // 2), (nx - 2, 1, nz - 2),
           (1, ny - 2, nz // 3)]
    with grid(n, zmarch_min=None):
        say("extreme", n, split)
        out = diffusion.forward(dev(T0), dev(Ci), nt, 1.0, dt, *d, split=split)
        got = np.array([out[k, j, i].item() for (i, j, k) in pts])
        assert torch.equal(out[:, :, 0], out[:, :, -2]) and torch.equal(out[:, :, -1], out[:, :, 1])
        assert torch.equal(out[0], out[-2]) and torch.equal(out[-1], out[1])
        del out
    ref = oracle.run_points(T0, Ci, nt, 1.0, dt, *d, pts)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
