"""FP16 stochastic rounding bit for bit: every stored FP16 value of a step
equals the rounding rule applied to the step's exact FP32 value with the
random word of its point, both computed here on the host from their
definitions: the PCG hash of Jarzynski & Olano (JCGT 2020) keyed on
(seed, counter), plane and pair of points, and in the FP16 normal range
truncation after adding the top 13 bits of the point's word below the FP16
ulp.  This pins the hash scheme and the gfx950 conversion instruction the
kernels use for it, in every kernel that stores FP16 points."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, say  # noqa: E402
from paper_2211_15716_amd import igg  # noqa: E402

M32 = np.uint64(0xFFFFFFFF)


def pcg_hash(v):
    """PCG hash (one LCG step, then the RXS-M-XS output permutation) of
    32-bit words, elementwise."""
    v = np.asarray(v, dtype=np.uint64) & M32
    state = (v * np.uint64(747796405) + np.uint64(2891336453)) & M32
    word = (((state >> ((state >> np.uint64(28)) + np.uint64(4))) ^ state) * np.uint64(277803737)) & M32
    return ((word >> np.uint64(22)) ^ word) & M32


def sr_key(seed, counter):
    """Key of a (seed, counter) pair: the hash chained over their four
    32-bit halves."""
    h = pcg_hash(counter >> 32)
    h = pcg_hash(np.uint64(counter & 0xFFFFFFFF) ^ h)
    h = pcg_hash(np.uint64(seed >> 32) ^ h)
    return pcg_hash(np.uint64(seed & 0xFFFFFFFF) ^ h)


def point_words(n, seed, counter, ol=(2, 2, 2)):
    """The random word of every point (k, j, i) of one rank on a periodic
    grid: plane key pcg(key + k), pair word pcg(plane key + i // 2 + gnh * j
    mod 2^32) with indices taken modulo the period; even i takes the word,
    odd i its low half moved to the top."""
    nx, ny, nz = n
    per = [d - o for d, o in zip(n, ol)]
    wrap = lambda g, p: np.where(g >= p, g - p, g)  # noqa: E731
    gi = wrap(np.arange(nx), per[0]).astype(np.uint64)
    gj = wrap(np.arange(ny), per[1]).astype(np.uint64)
    gk = wrap(np.arange(nz), per[2]).astype(np.uint64)
    key = sr_key(seed, counter)
    pk = pcg_hash((key + gk) & M32)
    gnh = np.uint64((nx + 1) // 2)
    pair = (gi[None, :] >> np.uint64(1)) + gnh * gj[:, None]
    w = pcg_hash((pk[:, None, None] + pair[None, :, :]) & M32)
    odd = (gi & np.uint64(1)).astype(bool)[None, None, :]
    return np.where(odd, (w << np.uint64(16)) & M32, w)


def round_rule(x32, w):
    """FP16 bits of float32 values x32 in the FP16 normal range rounded with
    words w: add the top 13 bits of w to the float's bits, clear the 13 bits
    an FP16 value does not have."""
    b = x32.view(np.uint32).astype(np.uint64)
    y = ((b + (w >> np.uint64(19))) & np.uint64(0xFFFFE000)).astype(np.uint32).view(np.float32)
    return y.astype(np.float16).view(np.uint16)


@pytest.mark.parametrize("nx,olx", [(70, 2), (72, 2), (72, 3)])
@pytest.mark.parametrize("split,zmin", [(None, 0), ((16, 2, 2), 0), (None, None), ((16, 2, 2), None)])
def test_fp16_stochastic_rounding_bits_match_their_definition(split, zmin, nx, olx):
    """Unsplit and boundary-first steps, on the z-march tiles (with the slab
    waves) and on the small-grid kernels.  Rows of 70 points take one point
    per lane, rows of 72 the kernels of 4-point vectors: with x overlap 2
    the period (70) is even and every vector holds two whole hash pairs
    (the vector at x = 68..71 straddles the period between its pairs); with
    overlap 3 the period (69) is odd and pairs straddle vectors."""
    n = (nx, 40, 36)
    ols = (olx, 2, 2)
    nx, ny, nz = n
    seed, counter = 0x1234_5678_9ABC, 7
    say("sr bits", split, zmin, nx, olx)
    rng = np.random.default_rng(5)
    T0 = 1.7 + 0.8 * rng.random((nz, ny, nx))
    Ci = 0.25 + 0.5 * rng.random((nz, ny, nx))
    dx = 1.0 / (nx - 1)
    dt = dx * dx / 0.75 / 6.1
    with grid(n, overlaps=ols, zmarch_min=zmin):
        T16, C16 = dev(T0, torch.float16), dev(Ci, torch.float16)
        exact = torch.empty(T16.shape, dtype=torch.float32, device="cuda")
        igg.diffusion_step(exact, T16.float().contiguous(), C16.float().contiguous(), 1.0, dt, dx, dx, dx,
                           split=split)
        out = torch.empty_like(T16)
        igg.diffusion_step(out, T16, C16, 1.0, dt, dx, dx, dx, split=split,
                           rnd=igg.rounding("stochastic", seed, counter))
        torch.cuda.synchronize()
        x = exact.cpu().numpy()[1:-1, 1:-1, 1:-1]
        got = out.cpu().numpy().view(np.uint16)[1:-1, 1:-1, 1:-1]
    ax = np.abs(x)
    assert np.all((ax >= 2.0 ** -14) & (ax < 65504.0))  # the normal range the rule covers
    w = point_words(n, seed, counter, ols)[1:-1, 1:-1, 1:-1]
    want = round_rule(np.ascontiguousarray(x), w)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} points differ, first (k, j, i) {tuple(bad[0])}"
    # and the rounding did something: both directions occur
    rn = x.astype(np.float16).view(np.uint16)
    assert np.any(got != rn)


def round_rule_all(x32, w):
    """FP16 bits of float32 values rounded with words w in every range: the
    normal range as above; below it (FP16 subnormals, spacing 2^-24) up with
    probability frac(|x| * 2^24), compared with the top 16 bits of w as a
    uniform in [0, 1); at or above 65504 to nearest."""
    ax = np.abs(x32)
    out = np.empty(x32.shape, np.uint16)
    normal = (ax >= np.float32(2.0 ** -14)) & (ax < np.float32(65504.0))
    sub = ax < np.float32(2.0 ** -14)
    big = ~normal & ~sub
    out[normal] = round_rule(np.ascontiguousarray(x32[normal]), w[normal])
    s = ax[sub] * np.float32(2.0 ** 24)
    f = np.floor(s)
    u = (w[sub] >> np.uint64(16)).astype(np.float32) * np.float32(2.0 ** -16)
    m = np.where(u < s - f, f + np.float32(1.0), f).astype(np.float32)
    out[sub] = np.copysign(m * np.float32(2.0 ** -24), x32[sub]).astype(np.float16).view(np.uint16)
    with np.errstate(over="ignore"):  # beyond 65520 the nearest FP16 value is infinity
        out[big] = x32[big].astype(np.float16).view(np.uint16)
    return out


@pytest.mark.parametrize("nx", [70, 72])
def test_fp16_stochastic_rounding_bits_from_subnormals_to_the_top_binade(nx):
    """The same check where the step's values fall in the subnormal range
    as well as the normal range: planes of FP16 subnormals, of ordinary
    values and of values just below the largest FP16 value, 65504 (a stable
    step is a convex combination of neighbours, so its results stay at or
    below 65504 and the range beyond it is not reached), and planes where
    each point draws its range at random, so that one vector of results
    mixes ranges."""
    n = (nx, 40, 36)
    nx, ny, nz = n
    seed, counter = 977, 3
    say("sr bits, every range", nx)
    rng = np.random.default_rng(9)
    T0 = np.empty((nz, ny, nx))
    T0[:8] = rng.uniform(1e-7, 5e-5, (8, ny, nx))
    T0[8:16] = rng.uniform(1.5, 2.5, (8, ny, nx))
    T0[16:24] = rng.uniform(65000.0, 65504.0, (8, ny, nx))
    pick = rng.integers(0, 3, (nz - 24, ny, nx))
    T0[24:] = np.choose(pick, [rng.uniform(1e-7, 5e-5, pick.shape), rng.uniform(1.5, 2.5, pick.shape),
                               rng.uniform(65000.0, 65504.0, pick.shape)])
    Ci = rng.uniform(0.25, 0.75, (nz, ny, nx))
    dx = 1.0 / (nx - 1)
    dt = dx * dx / 0.75 / 6.1
    with grid(n, zmarch_min=0):
        T16, C16 = dev(T0, torch.float16), dev(Ci, torch.float16)
        exact = torch.empty(T16.shape, dtype=torch.float32, device="cuda")
        igg.diffusion_step(exact, T16.float().contiguous(), C16.float().contiguous(), 1.0, dt, dx, dx, dx,
                           split=(16, 2, 2))
        out = torch.empty_like(T16)
        igg.diffusion_step(out, T16, C16, 1.0, dt, dx, dx, dx, split=(16, 2, 2),
                           rnd=igg.rounding("stochastic", seed, counter))
        torch.cuda.synchronize()
        x = exact.cpu().numpy()[1:-1, 1:-1, 1:-1]
        got = out.cpu().numpy().view(np.uint16)[1:-1, 1:-1, 1:-1]
    ax = np.abs(x)
    # subnormal results, ordinary ones and ones in the top FP16 binade occur
    assert np.any(ax < 2.0 ** -14) and np.any((ax >= 1.0) & (ax < 4.0)) and np.any(ax >= 32768.0)
    w = point_words(n, seed, counter)[1:-1, 1:-1, 1:-1]
    want = round_rule_all(np.ascontiguousarray(x), w)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} points differ, first (k, j, i) {tuple(bad[0])}"


@pytest.mark.parametrize("nx", [70, 72])
@pytest.mark.parametrize("split", [None, (16, 2, 2)])
def test_fp16_round_to_nearest_bits_match_the_fp32_step(split, nx):
    """Round-to-nearest FP16 stores: every stored value equals the step's
    FP32 value rounded to the nearest FP16 value (ties to even), in the
    kernels of one point per lane (70-point rows) and of 4-point vectors
    (72-point rows), unsplit and boundary-first."""
    n = (nx, 40, 36)
    nz, ny = n[2], n[1]
    say("rn bits", split, nx)
    rng = np.random.default_rng(11)
    T0 = 1.7 + 0.8 * rng.random((nz, ny, nx))
    Ci = 0.25 + 0.5 * rng.random((nz, ny, nx))
    dx = 1.0 / (nx - 1)
    dt = dx * dx / 0.75 / 6.1
    with grid(n, zmarch_min=0):
        T16, C16 = dev(T0, torch.float16), dev(Ci, torch.float16)
        exact = torch.empty(T16.shape, dtype=torch.float32, device="cuda")
        igg.diffusion_step(exact, T16.float().contiguous(), C16.float().contiguous(), 1.0, dt, dx, dx, dx,
                           split=split)
        out = torch.empty_like(T16)
        igg.diffusion_step(out, T16, C16, 1.0, dt, dx, dx, dx, split=split)
        torch.cuda.synchronize()
        x = exact.cpu().numpy()[1:-1, 1:-1, 1:-1]
        got = out.cpu().numpy().view(np.uint16)[1:-1, 1:-1, 1:-1]
    want = x.astype(np.float16).view(np.uint16)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} points differ, first (k, j, i) {tuple(bad[0])}"
