"""igg_reduce_noalloc, the reduction for callers that cannot allocate: through
the C ABI it gives igg_reduce's bits for every operation and element type, on
two calls in a row with the second on a smaller field (the static partial
results keep the first call's contents), and it allocates no device memory."""
import math

import numpy as np
import pytest

from paper_2211_15716_amd import igg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from gpu_common import grid, say  # noqa: E402

OPS = [igg.RED_MAX, igg.RED_MIN, igg.RED_SUM, igg.RED_SUM_RATIO, igg.RED_HALF_SQDIFF, igg.RED_DOT,
       igg.RED_MAX_ABS_DIFF, igg.RED_MAX_ABS]
DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}


def _noalloc(op, a, b, out):
    fa = igg.field(a)
    fb = igg.field(b)
    lib = igg.load()
    s = torch.cuda.current_stream()
    import ctypes
    rc = lib.igg_reduce_noalloc(int(op), ctypes.byref(fa), ctypes.byref(fb), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(s.cuda_stream))
    assert rc == igg.IGG_OK, lib.igg_last_error().decode()


@pytest.mark.parametrize("dt_name", ["f64", "f32", "f16"])
def test_noalloc_reduce_equals_reduce_on_two_calls(dt_name):
    results = []
    for n in ((96, 80, 70), (24, 20, 18)):  # the second call on a smaller field
        nx, ny, nz = n
        a_np, b_np = synth.uniform_fields(nx, ny, nz, seed=91 + nx, lo=0.5, hi=1.5, n=2)
        with grid(n):
            a = torch.from_numpy(a_np).cuda().to(DT[dt_name]).contiguous()
            b = torch.from_numpy(b_np).cuda().to(DT[dt_name]).contiguous()
            out = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            for op in OPS:
                say("noalloc", dt_name, n, op)
                ref = igg.reduce(op, a, b)
                torch.cuda.synchronize()
                before = torch.cuda.memory_allocated()
                _noalloc(op, a, b, out)
                torch.cuda.synchronize()
                assert torch.cuda.memory_allocated() == before
                got = out.item()
                assert got == ref or (math.isnan(got) and math.isnan(ref)), (op, got, ref)
                results.append((n, op, got))
        # the plain sum against an exactly rounded host sum
        inner = a_np[1:-1, 1:-1, 1:-1]
        if dt_name == "f64":
            exact = math.fsum(inner.ravel())
            s = [r for r in results if r[0] == n and r[1] == igg.RED_SUM][0][2]
            assert abs(s - exact) <= 1e-13 * abs(exact)
    assert len(results) == 2 * len(OPS)


def test_noalloc_reduce_rejects_bad_arguments():
    with grid((16, 12, 10)):
        a = torch.zeros((10, 12, 16), dtype=torch.float64, device="cuda")
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(igg.IggError):
            igg.reduce_noalloc(99, a, out)
        with pytest.raises(igg.IggError):
            igg.reduce_noalloc(igg.RED_DOT, a, out)  # DOT needs b
        bad = torch.zeros((10, 12, 15), dtype=torch.float64, device="cuda")
        with pytest.raises(igg.IggError):
            igg.reduce_noalloc(igg.RED_SUM, bad, out)
        igg.reduce_noalloc(igg.RED_SUM, a, out)
        torch.cuda.synchronize()
        assert out.item() == 0.0
