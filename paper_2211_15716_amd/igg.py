"""Python binding of the C-ABI library libigg_mi355x.so (include/igg.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors are torch tensors on the HIP device, contiguous, of shape
(nz, ny, nx) (x fastest), dtype float64, float32 or float16.  Calls are
ordered on torch's current stream unless a stream is passed.

The library is loaded on first use; if it is missing, every call raises
(there is no fallback path).  torch is imported first so that the library
binds to the HIP runtime torch has loaded.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libigg_mi355x.so")

IGG_OK = 0
IGG_ERR_STATE = -1
IGG_ERR_ARG = -2
IGG_ERR_SIZE = -3
IGG_ERR_DTYPE = -4
IGG_ERR_ALIAS = -5
IGG_ERR_HIP = -6

IGG_F64, IGG_F32, IGG_F16 = 0, 1, 2
IGG_ROUND_NEAREST, IGG_ROUND_STOCHASTIC = 0, 1

RED_MAX, RED_MIN, RED_SUM, RED_SUM_RATIO, RED_HALF_SQDIFF, RED_DOT, RED_MAX_ABS_DIFF, RED_MAX_ABS = range(8)
MAX_FIELDS = 8
MAX_RANKS = 64

EXPORTS = ["igg_init_global_grid", "igg_global_size", "igg_topology", "igg_update_halo",
           "igg_finalize_global_grid", "diffusion_step", "diffusion_dt", "diffusion_step_adjoint",
           "diffusion_flux_step", "diffusion_flux_step_adjoint", "igg_reduce", "igg_plan_split",
           "igg_timing_enable", "igg_timing_read", "igg_last_error", "igg_version",
           "igg_nranks", "igg_rank_coords", "igg_neighbors", "igg_update_halo_ranks", "diffusion_step_ranks",
           "diffusion_step_adjoint_ranks", "diffusion_flux_step_ranks", "diffusion_flux_step_adjoint_ranks",
           "diffusion_run", "igg_stream_probe", "igg_reduce_noalloc", "igg_adjoint_seed"]


class IggError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"igg error {code}: {msg}")
        self.code = code


class Field(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("size", ctypes.c_int64 * 3)]


class Rounding(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("counter", ctypes.c_uint64)]


_INT3 = ctypes.c_int * 3
_PI = ctypes.POINTER(ctypes.c_int)
_PF = ctypes.POINTER(Field)
_lib_handle = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or paper_2211_15716_amd/build.py)")
    import torch  # noqa: F401  -- binds the library to torch's HIP runtime
    lib = ctypes.CDLL(LIB_PATH)
    d, vp, i64p = ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    lib.igg_init_global_grid.argtypes = [ctypes.c_int] * 3 + [_PI, _PI, _PI, _PI]
    lib.igg_global_size.argtypes = [i64p]
    lib.igg_topology.argtypes = [_PI] * 5
    lib.igg_update_halo.argtypes = [_PF, ctypes.c_int, vp]
    lib.igg_update_halo_ranks.argtypes = [_PF, ctypes.c_int, vp]
    lib.igg_nranks.argtypes = [_PI]
    lib.igg_rank_coords.argtypes = [ctypes.c_int, _PI]
    lib.igg_neighbors.argtypes = [ctypes.c_int, _PI, _PI]
    lib.igg_finalize_global_grid.argtypes = []
    lib.diffusion_step.argtypes = [_PF] * 3 + [d] * 5 + [_PI, ctypes.POINTER(Rounding), vp]
    lib.diffusion_step_ranks.argtypes = [_PF] * 3 + [d] * 5 + [_PI, ctypes.POINTER(Rounding), vp]
    lib.diffusion_run.argtypes = [_PF] * 3 + [d] * 5 + [_PI, ctypes.POINTER(Rounding), ctypes.c_int, ctypes.c_int,
                                                        _PI, vp]
    lib.diffusion_dt.argtypes = [_PF, d, d, d, d, ctypes.POINTER(d), vp]
    lib.diffusion_step_adjoint.argtypes = [_PF] * 5 + [d] * 5 + [_PI, vp]
    lib.diffusion_step_adjoint_ranks.argtypes = [_PF] * 5 + [d] * 5 + [_PI, vp]
    lib.diffusion_flux_step_ranks.argtypes = [_PF] * 6 + [d] * 5 + [_PI, vp]
    lib.diffusion_flux_step_adjoint_ranks.argtypes = [_PF] * 5 + [d] * 5 + [_PI, vp]
    lib.diffusion_flux_step.argtypes = [_PF] * 6 + [d] * 5 + [_PI, vp]
    lib.diffusion_flux_step_adjoint.argtypes = [_PF] * 5 + [d] * 5 + [_PI, vp]
    lib.igg_reduce.argtypes = [ctypes.c_int, _PF, _PF, ctypes.POINTER(d), vp]
    lib.igg_reduce_noalloc.argtypes = [ctypes.c_int, _PF, _PF, vp, vp]
    lib.igg_adjoint_seed.argtypes = [_PF, _PF, _PF, ctypes.c_int, ctypes.POINTER(d), vp]
    lib.igg_plan_split.argtypes = [_PI, _PI, (ctypes.c_int * 6) * 7, _PI]
    lib.igg_timing_enable.argtypes = [ctypes.c_int]
    lib.igg_timing_read.argtypes = [ctypes.POINTER(d), i64p, i64p, ctypes.POINTER(d)]
    lib.igg_stream_probe.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int,
                                     ctypes.c_int64, vp]
    lib.igg_last_error.restype = ctypes.c_char_p
    lib.igg_version.restype = ctypes.c_char_p
    _lib_handle = lib
    return lib


def _check(rc):
    if rc != IGG_OK:
        raise IggError(rc, load().igg_last_error().decode())
    return rc


# ------------------------------------------------------------------ marshalling
def _dtype_code(t):
    import torch
    m = {torch.float64: IGG_F64, torch.float32: IGG_F32, torch.float16: IGG_F16}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def field(t):
    """igg_field of a contiguous (nz, ny, nx) device tensor."""
    if t.dim() != 3:
        raise ValueError("fields are 3-D tensors of shape (nz, ny, nx)")
    if not t.is_cuda:
        raise ValueError("fields must live on the HIP device")
    if not t.is_contiguous():
        raise ValueError("fields must be contiguous")
    nz, ny, nx = t.shape
    return Field(t.data_ptr(), _dtype_code(t), 0, (ctypes.c_int64 * 3)(nx, ny, nz))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _int3(v):
    return None if v is None else _INT3(*[int(x) for x in v])


# ------------------------------------------------------------------ grid
def init_global_grid(nx, ny, nz, dims=(0, 0, 0), periods=(0, 0, 0), overlaps=(2, 2, 2)):
    """Create the implicit global grid; returns the rank `me` (0)."""
    me = ctypes.c_int(-1)
    _check(load().igg_init_global_grid(int(nx), int(ny), int(nz), _int3(dims), _int3(periods),
                                       _int3(overlaps), ctypes.byref(me)))
    return me.value


def finalize_global_grid():
    _check(load().igg_finalize_global_grid())


def global_size():
    n = (ctypes.c_int64 * 3)()
    _check(load().igg_global_size(n))
    return tuple(n)


def nx_g():
    return global_size()[0]


def ny_g():
    return global_size()[1]


def nz_g():
    return global_size()[2]


def topology():
    arrs = [_INT3() for _ in range(5)]
    _check(load().igg_topology(*arrs))
    keys = ("n", "dims", "periods", "overlaps", "coords")
    return {k: tuple(a) for k, a in zip(keys, arrs)}


def update_halo(*tensors, stream=None):
    """Halo update of one or more fields (sizes n or n+1 per dimension)."""
    fs = (Field * len(tensors))(*[field(t) for t in tensors])
    _check(load().igg_update_halo(fs, len(tensors), _stream(stream)))


def nranks():
    """Ranks the grid holds (the product of dims; several = virtual ranks)."""
    n = ctypes.c_int(0)
    _check(load().igg_nranks(ctypes.byref(n)))
    return n.value


def rank_coords(rank):
    c = _INT3()
    _check(load().igg_rank_coords(int(rank), c))
    return tuple(c)


def neighbors(rank):
    """(lower, upper) neighbour ranks per dimension, -1 where there is none."""
    lo, hi = _INT3(), _INT3()
    _check(load().igg_neighbors(int(rank), lo, hi))
    return tuple(lo), tuple(hi)


def update_halo_ranks(*per_rank, stream=None):
    """Halo update across the grid's ranks: per_rank[r] is rank r's tuple of
    fields (the same number of fields for every rank)."""
    nf = len(per_rank[0])
    if any(len(fs) != nf for fs in per_rank):
        raise ValueError("every rank must pass the same number of fields")
    flat = [t for fs in per_rank for t in fs]
    arr = (Field * len(flat))(*[field(t) for t in flat])
    _check(load().igg_update_halo_ranks(arr, nf, _stream(stream)))


# ------------------------------------------------------------------ step
def rounding(mode="stochastic", seed=0, counter=0):
    code = {"nearest": IGG_ROUND_NEAREST, "stochastic": IGG_ROUND_STOCHASTIC}[mode]
    return Rounding(code, 0, int(seed), int(counter))


def diffusion_step(T2, T, Ci, lam, dt, dx, dy, dz, split=(16, 2, 2), rnd=None, stream=None):
    """One Fig. 1 step plus the halo update of T2 (boundary-first when split is given)."""
    f2, f, fc = field(T2), field(T), field(Ci)
    r = ctypes.byref(rnd) if rnd is not None else None
    _check(load().diffusion_step(ctypes.byref(f2), ctypes.byref(f), ctypes.byref(fc), float(lam), float(dt),
                                 float(dx), float(dy), float(dz), _int3(split), r, _stream(stream)))


def diffusion_step_ranks(T2s, Ts, Cis, lam, dt, dx, dy, dz, split=(16, 2, 2), rnd=None, stream=None):
    """diffusion_step on every rank's block (lists with one tensor per rank)."""
    P = len(Ts)
    a2 = (Field * P)(*[field(t) for t in T2s])
    a = (Field * P)(*[field(t) for t in Ts])
    ac = (Field * P)(*[field(t) for t in Cis])
    r = ctypes.byref(rnd) if rnd is not None else None
    _check(load().diffusion_step_ranks(a2, a, ac, float(lam), float(dt), float(dx), float(dy), float(dz),
                                       _int3(split), r, _stream(stream)))


def diffusion_step_adjoint_ranks(lam_ns, lam_np1s, T_ns, Cis, gCis, lam, dt, dx, dy, dz, split=(16, 2, 2),
                                 stream=None):
    """diffusion_step_adjoint on every rank's block (lists with one tensor per rank)."""
    arrs = [(Field * len(ts))(*[field(t) for t in ts]) for ts in (lam_ns, lam_np1s, T_ns, Cis, gCis)]
    _check(load().diffusion_step_adjoint_ranks(*arrs, float(lam), float(dt), float(dx), float(dy), float(dz),
                                               _int3(split), _stream(stream)))


def diffusion_flux_step_ranks(T2s, Ts, Cis, qxs, qys, qzs, lam, dt, dx, dy, dz, split=None, stream=None):
    """diffusion_flux_step on every rank's blocks (lists with one tensor per rank)."""
    arrs = [(Field * len(ts))(*[field(t) for t in ts]) for ts in (T2s, Ts, Cis, qxs, qys, qzs)]
    _check(load().diffusion_flux_step_ranks(*arrs, float(lam), float(dt), float(dx), float(dy), float(dz),
                                            _int3(split), _stream(stream)))


def diffusion_flux_step_adjoint_ranks(lam_ns, lam_np1s, T_ns, Cis, gCis, lam, dt, dx, dy, dz, split=None,
                                      stream=None):
    """diffusion_flux_step_adjoint on every rank's block."""
    arrs = [(Field * len(ts))(*[field(t) for t in ts]) for ts in (lam_ns, lam_np1s, T_ns, Cis, gCis)]
    _check(load().diffusion_flux_step_adjoint_ranks(*arrs, float(lam), float(dt), float(dx), float(dy),
                                                    float(dz), _int3(split), _stream(stream)))


def diffusion_run(T, T2, Ci, lam, dt, dx, dy, dz, nt, split=(16, 2, 2), rnd=None, graph=True, stream=None):
    """nt steps of the Fig. 1 time loop on the buffers T and T2 (swapped each
    step); with graph=True the library replays a captured HIP graph of two
    steps.  Returns the tensor holding the final state (T or T2)."""
    fb = ctypes.c_int(0)
    r = ctypes.byref(rnd) if rnd is not None else None
    f, f2, fc = field(T), field(T2), field(Ci)
    _check(load().diffusion_run(ctypes.byref(f), ctypes.byref(f2), ctypes.byref(fc), float(lam), float(dt), float(dx),
                                float(dy), float(dz), _int3(split), r, int(nt), 1 if graph else 0, ctypes.byref(fb),
                                _stream(stream)))
    return T2 if fb.value else T


def diffusion_dt(Ci, lam, dx, dy, dz, stream=None):
    out = ctypes.c_double()
    fc = field(Ci)
    _check(load().diffusion_dt(ctypes.byref(fc), float(lam), float(dx), float(dy), float(dz),
                               ctypes.byref(out), _stream(stream)))
    return out.value


def diffusion_step_adjoint(lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split=(16, 2, 2), stream=None):
    fs = [field(t) for t in (lam_n, lam_np1, T_n, Ci, gCi)]
    _check(load().diffusion_step_adjoint(*[ctypes.byref(f) for f in fs], float(lam), float(dt), float(dx),
                                         float(dy), float(dz), _int3(split), _stream(stream)))


def diffusion_flux_step(T2, T, Ci, qx, qy, qz, lam, dt, dx, dy, dz, split=None, stream=None):
    """Staggered flux form of the step plus the halo update of T2, qx, qy, qz
    (boundary-first when split is given; widths >= overlap + 1)."""
    fs = [field(t) for t in (T2, T, Ci, qx, qy, qz)]
    _check(load().diffusion_flux_step(*[ctypes.byref(f) for f in fs], float(lam), float(dt), float(dx),
                                      float(dy), float(dz), _int3(split), _stream(stream)))


def diffusion_flux_step_adjoint(lam_n, lam_np1, T_n, Ci, gCi, lam, dt, dx, dy, dz, split=None, stream=None):
    """Adjoint of the flux-form step n: lam_n from lam_np1 (valid halo), gCi
    accumulated; the fluxes of step n are formed from T_n."""
    fs = [field(t) for t in (lam_n, lam_np1, T_n, Ci, gCi)]
    _check(load().diffusion_flux_step_adjoint(*[ctypes.byref(f) for f in fs], float(lam), float(dt), float(dx),
                                              float(dy), float(dz), _int3(split), _stream(stream)))


# ------------------------------------------------------------------ reductions and helpers
def reduce(op, a, b=None, stream=None):
    fa = field(a)
    fb = field(b) if b is not None else None
    out = ctypes.c_double()
    _check(load().igg_reduce(int(op), ctypes.byref(fa), ctypes.byref(fb) if fb is not None else None,
                             ctypes.byref(out), _stream(stream)))
    return out.value


def adjoint_seed(lam, T=None, T_obs=None, halo=True, loss=False, stream=None):
    """lam = T - T_obs on the inner points (T alone without T_obs, zero
    without T), zero halo, then the halo update when halo is set; returns the
    FP64 loss 0.5*||T - T_obs||^2 over the inner points when loss is set
    (needs T_obs; synchronises), else None."""
    fl = field(lam)
    ft = field(T) if T is not None else None
    fo = field(T_obs) if T_obs is not None else None
    out = ctypes.c_double()
    _check(load().igg_adjoint_seed(ctypes.byref(ft) if ft is not None else None,
                                   ctypes.byref(fo) if fo is not None else None, ctypes.byref(fl),
                                   1 if halo else 0, ctypes.byref(out) if loss else None, _stream(stream)))
    return out.value if loss else None


def reduce_noalloc(op, a, out, b=None, stream=None):
    """reduce() into `out`, a one-element float64 device tensor, without
    allocating and without synchronising (igg_reduce_noalloc)."""
    import torch
    if out.dtype != torch.float64 or out.numel() != 1 or not out.is_cuda:
        raise ValueError("out must be a one-element float64 device tensor")
    fa = field(a)
    fb = field(b) if b is not None else None
    _check(load().igg_reduce_noalloc(int(op), ctypes.byref(fa), ctypes.byref(fb) if fb is not None else None,
                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)))


def plan_split(n, split):
    boxes = ((ctypes.c_int * 6) * 7)()
    nb = ctypes.c_int()
    _check(load().igg_plan_split(_int3(n), _int3(split), boxes, ctypes.byref(nb)))
    return [tuple(boxes[q]) for q in range(nb.value)]


def timing_enable(on=True):
    _check(load().igg_timing_enable(1 if on else 0))


def timing_read():
    """(inner ms, inner launches, inner points, boundary ms) since the last read."""
    ms = ctypes.c_double()
    bms = ctypes.c_double()
    launches = ctypes.c_int64()
    points = ctypes.c_int64()
    _check(load().igg_timing_read(ctypes.byref(ms), ctypes.byref(launches), ctypes.byref(points),
                                  ctypes.byref(bms)))
    return ms.value, launches.value, points.value, bms.value


def stream_probe(srcs, dsts, stream=None):
    """dst = sum of srcs for every dst (FP64 device tensors of one size): the
    streaming probe of the given read/write mix."""
    n = srcs[0].numel()
    for t in list(srcs) + list(dsts):
        if t.dtype.itemsize != 8 or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("probe arrays are contiguous 8-byte device tensors of one size")
    sa = (ctypes.c_void_p * len(srcs))(*[t.data_ptr() for t in srcs])
    da = (ctypes.c_void_p * len(dsts))(*[t.data_ptr() for t in dsts])
    _check(load().igg_stream_probe(sa, len(srcs), da, len(dsts), n, _stream(stream)))


def version():
    return load().igg_version().decode()
