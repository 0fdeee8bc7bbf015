"""Overlap must not change results (Sec. 2: the boundary and the halo update
run beside the inner region): translation equivariance on the periodic grid,
a held-back stream on either side of the boundary-first schedule, the slab
kernel's fused pack against the separate halo pass, and the copies of one
physical point under overlaps above 2 rounding alike in FP16 with
stochastic rounding."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, inner, say  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def _shift_unique(A, s):
    """The field whose unique (inner) points are A's rolled by s = (sx, sy,
    sz) points, with the periodic halo of overlap 2 applied."""
    out = A.copy()
    inner(out)[...] = np.roll(inner(A), shift=(s[2], s[1], s[0]), axis=(0, 1, 2))
    oracle.halo(out)
    return out


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_translation_equivariance(dt_name):
    """Shifting T0 and Ci by s on the periodic grid shifts the result by s,
    bit for bit (FP16 with round-to-nearest stores), unsplit and
    boundary-first.  The grid spans several x tiles of every precision,
    several tile rows and z chunks, with the XCD-aware work-group order
    active; the shift crosses tile, chunk and slab boundaries."""
    n = (300, 70, 52)
    s = (131, 17, 9)
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=81, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    T0s, Cis = _shift_unique(T0, s), _shift_unique(Ci, s)
    d = (1 / 299, 1 / 69, 1 / 51)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    with grid(n):
        for split in (None, (16, 2, 2), (16, 5, 3)):
            say("translation", dt_name, split)
            a = host(diffusion.forward(dev(T0, DT[dt_name]), dev(Ci, DT[dt_name]), 6, 1.0, dt, *d, split=split))
            b = host(diffusion.forward(dev(T0s, DT[dt_name]), dev(Cis, DT[dt_name]), 6, 1.0, dt, *d, split=split))
            assert np.array_equal(inner(b), np.roll(inner(a), shift=(s[2], s[1], s[0]), axis=(0, 1, 2)))
            assert np.array_equal(b, oracle.halo(b.copy()))


@pytest.mark.parametrize("where", ["side:300", "inner:300", "halo:300"])
@pytest.mark.parametrize("pack", ["1", "2", "0"])
def test_held_back_stream_gives_same_bits(where, pack, monkeypatch):
    """A fixed wait of about a millisecond (longer than a step here) put into
    the helper stream before the slabs, into the caller stream before the
    inner region, or before the halo update: every schedule, eager and in
    the library's captured time loop, gives the serial chain's bits."""
    n = (260, 140, 72)  # inner region above 2^21 points: the helper stream is used by default
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=83, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    d = (1 / 259, 1 / 139, 1 / 71)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    nt = 7
    monkeypatch.setenv("IGG_SLAB_PACK", pack)
    monkeypatch.setenv("IGG_SCHEDULE", "2")
    with grid(n, zmarch_min=None):
        ref = host(diffusion.forward(dev(T0), dev(Ci), nt, 1.0, dt, *d, split=(16, 2, 2)))
    monkeypatch.setenv("IGG_TEST_DELAY", where)
    for sched in ("1", "0", "2", "3"):
        monkeypatch.setenv("IGG_SCHEDULE", sched)
        with grid(n, zmarch_min=None):
            say("held back", where, "pack", pack, "schedule", sched)
            got = host(diffusion.forward(dev(T0), dev(Ci), nt, 1.0, dt, *d, split=(16, 2, 2)))
            assert np.array_equal(got, ref)
            T, W = dev(T0), dev(T0)
            fin = igg.diffusion_run(T, W, dev(Ci), 1.0, dt, *d, nt, split=(16, 2, 2), graph=True)
            assert np.array_equal(host(fin), ref)


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
@pytest.mark.parametrize("ol,split", [((2, 2, 2), (16, 2, 2)), ((3, 3, 3), (16, 4, 3)), ((2, 3, 4), (5, 3, 4))])
def test_fused_pack_equals_separate_halo_pass(dt_name, ol, split, monkeypatch):
    """The boundary-slab kernel packing the y and z planes (and their halo
    entries' images) with one exchange-and-unpack copy, or storing them
    straight into the halo planes, gives the bits of the separate pack,
    exchange and unpack passes, halos included, with the slabs on the helper
    stream, before the inner region on the caller stream, or in the inner
    region's launch."""
    n = (132, 40, 36)
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=85, noise=1e-2)
    oracle.halo(T0, ol)
    oracle.halo(Ci, ol)
    d = (1 / 131, 1 / 39, 1 / 35)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    outs = []
    for pack in ("1", "2", "0"):
        for sched in ("1", "2", "3"):
            monkeypatch.setenv("IGG_SLAB_PACK", pack)
            monkeypatch.setenv("IGG_SCHEDULE", sched)
            with grid(n, overlaps=ol):
                say("pack", pack, "schedule", sched, dt_name, ol, split)
                o = diffusion.forward(dev(T0, DT[dt_name]), dev(Ci, DT[dt_name]), 5, 1.0, dt, *d, split=split,
                                      sr_seed=5 if dt_name == "f16" else None)
                outs.append(host(o))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = oracle.run(T0, Ci, 5, 1.0, dt, *d, ol=ol)
    tol = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}[dt_name]
    assert np.max(np.abs(outs[0] - ref)) <= tol * np.max(np.abs(ref))


def test_fp16_stochastic_rounding_keeps_overlap_copies_equal():
    """With overlaps of 3 on a periodic grid, inner points 1 and n-2 of each
    dimension are one physical point computed twice; with stochastic
    rounding both copies draw the same random bits, so they stay bit-equal
    step after step (and the halo planes equal their images)."""
    n = (70, 38, 30)
    ol = (3, 3, 3)
    # fields of period n-ol in every dimension, so that the copies agree
    # from the start: local index l holds the value of global point l mod (n-ol)
    per = tuple(m - o for m, o in zip(n, ol))
    Tg, Cg = synth.noisy_state_uniform_ci(*per, seed=87, noise=1e-2)
    idx = np.ix_(*[np.arange(m) % p for m, p in zip(n[::-1], per[::-1])])
    T0, Ci = np.ascontiguousarray(Tg[idx]), np.ascontiguousarray(Cg[idx])
    assert np.array_equal(T0, oracle.halo(T0.copy(), ol))
    d = (1 / 69, 1 / 37, 1 / 29)
    dt = oracle.time_step(*d, 1.0, oracle.max_all(Ci))
    with grid(n, overlaps=ol):
        for split in (None, (16, 4, 3)):
            say("fp16 SR overlap copies", split)
            o = host(diffusion.forward(dev(T0, torch.float16), dev(Ci, torch.float16), 8, 1.0, dt, *d,
                                       split=split, sr_seed=3))
            assert np.array_equal(o[:, :, 1], o[:, :, -2])
            assert np.array_equal(o[:, 1, :], o[:, -2, :])
            assert np.array_equal(o[1, :, :], o[-2, :, :])
            assert np.array_equal(o, oracle.halo(o.copy(), ol))
