"""HIP-graph capture of the step chain (replays give the eager bits) and the
library's kernel timing events."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, say  # noqa: E402


@pytest.mark.parametrize("n,split,sched", [((32, 32, 32), (16, 2, 2), None), ((66, 40, 36), (16, 2, 2), None),
                                           ((48, 40, 36), None, None), ((66, 40, 36), (16, 2, 2), "1"),
                                           ((66, 40, 36), (16, 2, 2), "0"), ((66, 40, 36), (16, 2, 2), "2"),
                                           ((160, 140, 120), (16, 2, 2), None), ((160, 140, 120), (16, 2, 2), "1")])
def test_graph_replay_matches_eager(n, split, sched, monkeypatch):
    """Every schedule is capturable: the helper-stream forms (1, and 0)
    capture their fork and join events as graph edges; the one-launch form
    (3, the default for these one-rank periodic grids) and the serial chain
    (2) capture as a chain."""
    if sched is not None:
        monkeypatch.setenv("IGG_SCHEDULE", sched)
    say("graph", n, split, sched)
    w = synth.noisy_state_uniform_ci(*n, seed=71, noise=1e-2)
    T0, Ci = w
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1 / (n[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    pairs, reps = 2, 3
    with grid(n):
        C = dev(Ci)
        eager = diffusion.forward(dev(T0), C, 2 * pairs * reps, 1.0, dt, dx, dx, dx, split=split)
        ref = host(eager)
        T = dev(T0)
        T2 = T.clone()
        g = diffusion.StepGraph(T, T2, C, 1.0, dt, dx, dx, dx, split=split, pairs=pairs)
        for r in range(reps):
            g.replay()
            torch.cuda.synchronize()
            # eager work between replays must not disturb them
            junk = torch.ones(1000, device="cuda").sum().item()
            assert junk == 1000.0
        got = host(T)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,split,dt_name", [((32, 32, 32), (16, 2, 2), "f64"), ((66, 40, 36), (16, 2, 2), "f32"),
                                             ((48, 40, 36), None, "f64"), ((160, 140, 120), (16, 2, 2), "f64"),
                                             ((40, 34, 30), (16, 2, 2), "f16")])
def test_native_graph_run_matches_eager(n, split, dt_name):
    """diffusion_run with the library's captured graph equals eager steps bit
    for bit, for odd and even step counts, on repeated calls (the kept graph),
    after the arguments change (a new capture), with eager torch work between
    calls; FP16 with round-to-nearest stores."""
    say("native graph", n, split, dt_name)
    dt_map = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
    T0, Ci = synth.noisy_state_uniform_ci(*n, seed=73, noise=1e-2)
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1 / (n[0] - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    wdt = dt_map[dt_name]
    with grid(n, zmarch_min=None):
        C = dev(Ci, wdt)
        for nt in (1, 4, 7, 6, 37, 16):
            ref = host(diffusion.forward(dev(T0, wdt), C, nt, 1.0, dt, dx, dx, dx, split=split))
            for rep in range(2):
                T = dev(T0, wdt)
                T2 = T.clone()
                out = igg.diffusion_run(T, T2, C, 1.0, dt, dx, dx, dx, nt, split=split, graph=True)
                assert torch.ones(100, device="cuda").sum().item() == 100.0
                assert np.array_equal(host(out), ref), (nt, rep)
        # a different time step: the kept graph must be rebuilt
        ref = host(diffusion.forward(dev(T0, wdt), C, 4, 1.0, 0.5 * dt, dx, dx, dx, split=split))
        T = dev(T0, wdt)
        out = igg.diffusion_run(T, T.clone(), C, 1.0, 0.5 * dt, dx, dx, dx, 4, split=split, graph=True)
        assert np.array_equal(host(out), ref)
        if dt_name == "f16":
            with pytest.raises(igg.IggError):
                igg.diffusion_run(T, T.clone(), C, 1.0, dt, dx, dx, dx, 4, split=split,
                                  rnd=igg.rounding("stochastic", 1, 0), graph=True)
            # without the graph, stochastic rounding advances the counter per step
            sr = host(diffusion.forward(dev(T0, wdt), C, 5, 1.0, dt, dx, dx, dx, split=split, sr_seed=9))
            T = dev(T0, wdt)
            out = igg.diffusion_run(T, T.clone(), C, 1.0, dt, dx, dx, dx, 5, split=split,
                                    rnd=igg.rounding("stochastic", 9, 0), graph=False)
            assert np.array_equal(host(out), sr)


@pytest.mark.parametrize("split", [(4, 3, 3), None])
@pytest.mark.parametrize("sched", ["1", "3"])
def test_kernel_timing_events_count_launches_and_points(split, sched, monkeypatch):
    """The library's kernel timing (the figures the benchmark's roofline
    takes): with timing on, each step adds one inner launch of the expected
    number of points (in the one-launch schedule the slabs' points too) and
    a positive duration; a read resets the totals; more launches than the
    pre-made event pool grow it; with timing off nothing is counted; and
    timing does not change a result bit."""
    monkeypatch.setenv("IGG_SCHEDULE", sched)
    n = (40, 36, 34)
    nx, ny, nz = n
    rng = np.random.default_rng(71)
    T0 = rng.uniform(1.0, 2.0, (nz, ny, nx))
    Ci = rng.uniform(0.5, 1.5, (nz, ny, nx))
    oracle.halo(T0)
    oracle.halo(Ci)
    dx = 1.0 / (nx - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    side = split is not None and sched == "1"
    if not side:  # everything in the one launch
        pts = (nx - 2) * (ny - 2) * (nz - 2)
    else:  # x slabs join the inner launch; y and z slabs are the boundary
        pts = (nx - 2) * (ny - 2 * split[1]) * (nz - 2 * split[2])
    with grid(n):
        say("timing", split)
        T, C = dev(T0), dev(Ci)
        ref = diffusion.forward(T.clone(), C, 6, 1.0, dt, dx, dx, dx, split=split)
        igg.timing_enable(True)
        out = diffusion.forward(T.clone(), C, 6, 1.0, dt, dx, dx, dx, split=split)
        ms, launches, points, bms = igg.timing_read()
        assert torch.equal(out, ref)
        assert launches == 6 and points == 6 * pts
        assert ms > 0.0
        assert (bms > 0.0) == side
        assert igg.timing_read() == (0.0, 0, 0, 0.0)
        # more timed launches than the 2048 events made up front
        diffusion.forward(T.clone(), C, 1100, 1.0, dt, dx, dx, dx, split=split)
        ms, launches, points, bms = igg.timing_read()
        assert launches == 1100 and points == 1100 * pts and ms > 0.0
        igg.timing_enable(False)
        diffusion.forward(T.clone(), C, 3, 1.0, dt, dx, dx, dx, split=split)
        assert igg.timing_read() == (0.0, 0, 0, 0.0)
