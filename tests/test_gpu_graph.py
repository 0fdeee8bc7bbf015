"""HIP-graph capture of the step chain: replays give the eager bits."""
import numpy as np
import pytest

import oracle
from paper_2211_15716_amd import diffusion, igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import dev, grid, host, say  # noqa: E402


@pytest.mark.parametrize("n,split,sched", [((32, 32, 32), (16, 2, 2), None), ((66, 40, 36), (16, 2, 2), None),
                                           ((48, 40, 36), None, None), ((66, 40, 36), (16, 2, 2), "1"),
                                           ((66, 40, 36), (16, 2, 2), "0"), ((160, 140, 120), (16, 2, 2), None)])
def test_graph_replay_matches_eager(n, split, sched, monkeypatch):
    """Every schedule is capturable: the helper-stream forms (1, and 0)
    capture their fork and join events as graph edges; 160x140x120 takes
    schedule 1 by default."""
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
