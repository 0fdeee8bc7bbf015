"""Host-side tests of the C-ABI library: it loads, exports every function
include/igg.h declares, validates arguments before any HIP call, and its
host logic (global grid size, boundary-first partition) is right.

Calls here never reach a kernel: every call either fails validation or is a
pure host function.  The validation cases run only where no GPU is visible,
so their fake device pointers can never reach a HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2211_15716_amd import igg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char \*|double)\s*\*?\s*(\w+)\s*\(", src)))


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


no_gpu = pytest.mark.skipif(_gpu_visible(), reason="fake device pointers are only passed where no GPU exists")


def test_library_exports_every_declared_symbol():
    lib = igg.load()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(igg.EXPORTS)
    assert "gfx950" in igg.version()


@pytest.fixture
def host_grid():
    lib = igg.load()
    yield lib
    if igg.load().igg_topology(None, None, None, None, None) == 0:
        igg.load().igg_finalize_global_grid()


def _field(ptr, dtype, n):
    return igg.Field(ptr, dtype, 0, (ctypes.c_int64 * 3)(*n))


def test_grid_lifecycle_and_global_size(host_grid):
    lib = host_grid
    I3 = ctypes.c_int * 3
    n_g = (ctypes.c_int64 * 3)()
    assert lib.igg_global_size(n_g) == igg.IGG_ERR_STATE
    assert lib.igg_finalize_global_grid() == igg.IGG_ERR_STATE
    me = ctypes.c_int(-1)
    assert lib.igg_init_global_grid(512, 512, 512, None, None, None, ctypes.byref(me)) == 0
    assert me.value == 0
    assert lib.igg_global_size(n_g) == 0 and tuple(n_g) == (512, 512, 512)  # Fig. 1 defaults
    assert lib.igg_init_global_grid(8, 8, 8, None, None, None, None) == igg.IGG_ERR_STATE
    assert lib.igg_finalize_global_grid() == 0
    assert lib.igg_init_global_grid(32, 20, 12, I3(0, 1, 0), I3(1, 0, 1), I3(2, 3, 4), None) == 0
    assert lib.igg_global_size(n_g) == 0 and tuple(n_g) == (30, 20, 8)
    top = igg.topology()
    assert top == {"n": (32, 20, 12), "dims": (1, 1, 1), "periods": (1, 0, 1), "overlaps": (2, 3, 4),
                   "coords": (0, 0, 0)}
    assert lib.igg_finalize_global_grid() == 0


@pytest.mark.parametrize("args", [
    (2, 8, 8, None, None, None),                      # n < ol + 1
    (8, 8, 8, (8, 4, 4), None, None),                 # more virtual ranks than IGG_MAX_RANKS
    (8, 8, 8, None, (2, 0, 0), None),                 # period not 0/1
    (8, 8, 8, None, None, (1, 2, 2)),                 # overlap < 2
    (8, 8, 8, (-1, 1, 1), None, None),
    (5, 8, 8, None, None, (5, 2, 2)),
])
def test_init_rejects_bad_arguments(host_grid, args):
    lib = host_grid
    I3 = ctypes.c_int * 3
    nx, ny, nz, d, p, o = args
    cv = lambda v: None if v is None else I3(*v)  # noqa: E731
    assert lib.igg_init_global_grid(nx, ny, nz, cv(d), cv(p), cv(o), None) == igg.IGG_ERR_ARG
    assert lib.igg_last_error()


@no_gpu
def test_step_validation_before_any_hip_call(host_grid):
    lib = host_grid
    I3 = ctypes.c_int * 3
    assert lib.igg_init_global_grid(16, 12, 10, None, I3(1, 1, 1), None, None) == 0
    n = (16, 12, 10)
    T = _field(0x10000000, igg.IGG_F64, n)
    T2 = _field(0x20000000, igg.IGG_F64, n)
    C = _field(0x30000000, igg.IGG_F64, n)
    r = ctypes.byref
    step = lambda a, b, c, split=None, lam=1.0, dt=1e-3, rnd=None: lib.diffusion_step(  # noqa: E731
        r(a), r(b), r(c), lam, dt, 0.1, 0.1, 0.1, split, rnd, None)
    assert step(T, T, C) == igg.IGG_ERR_ALIAS
    assert step(T2, T, _field(0x20000008, igg.IGG_F64, n)) == igg.IGG_ERR_ALIAS
    assert step(_field(0x20000000, igg.IGG_F32, n), T, C) == igg.IGG_ERR_DTYPE
    assert step(_field(0x20000000, 7, n), T, C) == igg.IGG_ERR_DTYPE
    assert step(_field(0x20000000, igg.IGG_F64, (17, 12, 10)), T, C) == igg.IGG_ERR_SIZE
    assert step(_field(0, igg.IGG_F64, n), T, C) == igg.IGG_ERR_ARG
    assert step(T2, T, C, split=I3(16, 1, 2)) == igg.IGG_ERR_ARG
    assert step(T2, T, C, split=I3(-3, 2, 2)) == igg.IGG_ERR_ARG
    assert step(T2, T, C, lam=0.0) == igg.IGG_ERR_ARG
    assert step(T2, T, C, dt=float("nan")) == igg.IGG_ERR_ARG
    assert step(T2, T, C, rnd=r(igg.Rounding(5, 0, 0, 0))) == igg.IGG_ERR_ARG
    bad = igg.Field(0x20000000, igg.IGG_F64, 1, (ctypes.c_int64 * 3)(*n))
    assert step(bad, T, C) == igg.IGG_ERR_ARG
    # halo: staggered sizes accepted by validation, others refused
    fs = (igg.Field * 2)(_field(0x10000000, igg.IGG_F64, (18, 12, 10)), T2)
    assert lib.igg_update_halo(fs, 2, None) == igg.IGG_ERR_SIZE
    fs = (igg.Field * 2)(T, T)
    assert lib.igg_update_halo(fs, 2, None) == igg.IGG_ERR_ALIAS
    assert lib.igg_update_halo(fs, 0, None) == igg.IGG_ERR_ARG
    assert lib.igg_update_halo(fs, igg.MAX_FIELDS + 1, None) == igg.IGG_ERR_ARG
    # adjoint: FP16 refused, aliasing refused
    H = [_field(0x10000000 * (q + 1), igg.IGG_F16, n) for q in range(5)]
    assert lib.diffusion_step_adjoint(*[r(h) for h in H], 1.0, 1e-3, .1, .1, .1, None, None) == igg.IGG_ERR_DTYPE
    A = [_field(0x10000000 * (q + 1), igg.IGG_F64, n) for q in range(5)]
    A[4] = A[1]
    assert lib.diffusion_step_adjoint(*[r(a) for a in A], 1.0, 1e-3, .1, .1, .1, None, None) == igg.IGG_ERR_ALIAS
    # flux form: face sizes checked
    q = [_field(0x40000000 + 0x1000000 * d, igg.IGG_F64, n) for d in range(3)]
    assert lib.diffusion_flux_step(r(T2), r(T), r(C), *[r(x) for x in q], 1.0, 1e-3, .1, .1, .1,
                                   None, None) == igg.IGG_ERR_SIZE
    # flux form: split widths must cover the face fields' overlap ol + 1
    qf = [_field(0x40000000 + 0x1000000 * d, igg.IGG_F64, tuple(m + (e == d) for e, m in enumerate(n)))
          for d in range(3)]
    I3s = ctypes.c_int * 3
    assert lib.diffusion_flux_step(r(T2), r(T), r(C), *[r(x) for x in qf], 1.0, 1e-3, .1, .1, .1,
                                   I3s(16, 2, 2), None) == igg.IGG_ERR_ARG
    # flux form and its adjoint: FP16 refused
    h16 = [_field(0x60000000 + 0x1000000 * d, igg.IGG_F16, n) for d in range(3)]
    qh = [_field(0x70000000 + 0x1000000 * d, igg.IGG_F16, tuple(m + (e == d) for e, m in enumerate(n)))
          for d in range(3)]
    assert lib.diffusion_flux_step(*[r(x) for x in h16], *[r(x) for x in qh], 1.0, 1e-3, .1, .1, .1,
                                   None, None) == igg.IGG_ERR_DTYPE
    assert lib.diffusion_flux_step_adjoint(*[r(h) for h in H], 1.0, 1e-3, .1, .1, .1, None,
                                           None) == igg.IGG_ERR_DTYPE
    # reductions
    out = ctypes.c_double()
    assert lib.igg_reduce(99, r(T), None, r(out), None) == igg.IGG_ERR_ARG
    assert lib.igg_reduce(igg.RED_DOT, r(T), None, r(out), None) == igg.IGG_ERR_ARG
    assert lib.igg_reduce(igg.RED_DOT, r(T), r(_field(0x50000000, igg.IGG_F32, n)), r(out),
                          None) == igg.IGG_ERR_DTYPE
    assert lib.igg_finalize_global_grid() == 0


@no_gpu
def test_valid_call_without_gpu_reports_hip_error(host_grid):
    lib = host_grid
    I3 = ctypes.c_int * 3
    assert lib.igg_init_global_grid(16, 12, 10, None, I3(1, 1, 1), None, None) == 0
    n = (16, 12, 10)
    fs = (igg.Field * 1)(_field(0x10000000, igg.IGG_F64, n))
    assert lib.igg_update_halo(fs, 1, None) == igg.IGG_ERR_HIP
    assert "HIP" in lib.igg_last_error().decode()
    assert lib.igg_finalize_global_grid() == 0


@pytest.mark.parametrize("n,split", [((512, 512, 512), (16, 2, 2)), ((32, 32, 32), (16, 2, 2)),
                                     ((9, 7, 5), (2, 2, 2)), ((40, 30, 20), (3, 15, 10)),
                                     ((20, 20, 20), (19, 2, 3)), ((3, 3, 3), (2, 2, 2))])
def test_split_plan_partitions_inner_points(n, split):
    boxes = igg.plan_split(n, split)
    inner_box = boxes[-1]
    cover = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    for (i0, i1, j0, j1, k0, k1) in boxes:
        cover[k0:k1, j0:j1, i0:i1] += 1
    assert np.all(cover[1:-1, 1:-1, 1:-1] == 1)  # disjoint, and every inner point once
    assert cover.sum() == np.prod([m - 2 for m in n])
    # the boundary boxes hold every point within `split` of an array edge,
    # which includes both send planes (index 1 and n-2) of each dimension
    i0, i1, j0, j1, k0, k1 = inner_box
    if i0 < i1 and j0 < j1 and k0 < k1:
        assert (i0, j0, k0) == tuple(min(s, m - 1) for s, m in zip(split, n))
        assert (n[0] - i1, n[1] - j1, n[2] - k1) == tuple(s for s in split)
        assert i0 > 1 and j0 > 1 and k0 > 1
    if n == (512, 512, 512):
        assert inner_box == (16, 496, 2, 510, 2, 510)


@pytest.mark.parametrize("dims,periods", [((2, 3, 2), (1, 0, 1)), ((1, 1, 4), (0, 0, 1)), ((3, 1, 1), (0, 1, 0)),
                                          ((2, 2, 2), (1, 1, 1))])
def test_virtual_ranks_topology(host_grid, dims, periods):
    """Rank coordinates (x fastest) and neighbours against a brute force over
    the Cartesian topology; the global size against the oracle's formula."""
    import oracle
    n, ol = (10, 8, 7), (2, 3, 2)
    igg.init_global_grid(*n, dims=dims, periods=periods, overlaps=ol)
    try:
        P = dims[0] * dims[1] * dims[2]
        assert igg.nranks() == P
        assert igg.global_size() == tuple(oracle.global_size(n, dims, periods, ol))
        coords = {}
        for cz in range(dims[2]):
            for cy in range(dims[1]):
                for cx in range(dims[0]):
                    coords[len(coords)] = (cx, cy, cz)
        inv = {c: r for r, c in coords.items()}
        for r in range(P):
            assert igg.rank_coords(r) == coords[r]
            lo, hi = igg.neighbors(r)
            for d in range(3):
                for side, got in ((-1, lo[d]), (1, hi[d])):
                    c = list(coords[r])
                    c[d] += side
                    if 0 <= c[d] < dims[d]:
                        want = inv[tuple(c)]
                    elif periods[d]:
                        c[d] %= dims[d]
                        want = inv[tuple(c)]
                    else:
                        want = -1
                    assert got == want, (r, d, side)
        with pytest.raises(igg.IggError):
            igg.rank_coords(P)
        if P > 1:
            # the single-block entry points refuse a grid of several ranks
            # (a state check made before any argument is looked at)
            lib = igg.load()
            assert lib.diffusion_step(None, None, None, 1.0, 1e-3, 0.1, 0.1, 0.1, None, None, None) == \
                igg.IGG_ERR_STATE
            assert lib.igg_update_halo(None, 1, None) == igg.IGG_ERR_STATE
    finally:
        igg.finalize_global_grid()


def test_virtual_ranks_cover_the_global_grid():
    """The blocks' global index ranges c*(n-ol) + [0, n) tile the global
    index space 0 .. dims*(n-ol)+ol-1: neighbouring blocks share exactly ol
    indices and together they cover every index (the decomposition the GPU
    tests compare against one block of the global size)."""
    import oracle
    for n, ol, dims, per in [(10, 2, 3, 1), (9, 3, 2, 0), (12, 4, 4, 1), (5, 2, 1, 1)]:
        N = dims * (n - ol) + ol
        cover = np.zeros(N, int)
        for c in range(dims):
            cover[c * (n - ol): c * (n - ol) + n] += 1
        assert cover.min() >= 1 and cover.max() <= 2
        assert (cover == 2).sum() == (dims - 1) * ol
        # unique points: N minus the ol periodic images when periodic
        assert N - ol * per == oracle.global_size((n, n, n), (dims, 1, 1), (per, 0, 0), (ol, ol, ol))[0]


def test_rank_solvers_check_block_count_and_overlaps(host_grid):
    """DiffusionSolveRanks and loss_and_grad_ranks refuse, before any GPU
    work, a block count other than 2 x nranks and overlaps other than 2 (with
    wider overlaps the blocks' inner points share points, so a loss over
    them would count some unique points twice)."""
    torch = pytest.importorskip("torch")
    from paper_2211_15716_amd import diffusion
    t = torch.zeros(1)
    igg.init_global_grid(10, 8, 7, dims=(2, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2))
    try:
        with pytest.raises(ValueError, match="expected 4 blocks"):
            diffusion.DiffusionSolveRanks.apply(None, 2, ("store_all",), t, t, t)
    finally:
        igg.finalize_global_grid()
    igg.init_global_grid(10, 8, 7, dims=(2, 1, 1), periods=(1, 1, 1), overlaps=(3, 2, 2))
    try:
        with pytest.raises(ValueError, match="overlaps"):
            diffusion.DiffusionSolveRanks.apply(None, 2, ("store_all",), t, t, t, t)
        with pytest.raises(ValueError, match="overlaps"):
            diffusion.loss_and_grad_ranks([t, t], [t, t], [t, t], None, 2)
    finally:
        igg.finalize_global_grid()


@no_gpu
def test_stream_probe_validates_before_any_hip_call():
    """The streaming probe refuses bad counts, null and misaligned pointers
    on the host; zero elements launch nothing."""
    lib = igg.load()
    VP = ctypes.c_void_p
    ok = (VP * 4)(0x10000000, 0x10001000, 0x10002000, 0x10003000)
    bad = (VP * 1)(0x10000008 + 4)
    null = (VP * 1)(None)
    assert lib.igg_stream_probe(ok, 0, ok, 1, 16, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(ok, 5, ok, 1, 16, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(ok, 1, ok, 5, 16, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(ok, 2, ok, 1, 15, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(bad, 1, ok, 1, 16, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(null, 1, ok, 1, 16, None) == igg.IGG_ERR_ARG
    assert lib.igg_stream_probe(None, 1, ok, 1, 16, None) == igg.IGG_ERR_ARG
    lib.igg_stream_probe(bad, 1, ok, 1, 16, None)
    assert "aligned" in lib.igg_last_error().decode()
    assert lib.igg_stream_probe(ok, 2, ok, 2, 0, None) == igg.IGG_OK
