"""CPU FP64 oracle of the explicit 3-D diffusion step and its halo update.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP path; the arithmetic lives in ``oracle.c`` (plain loops,
FP64, the operation order of the paper's Fig. 1, no fused multiply-add) and
this module only marshals numpy arrays and strings together the time loop,
the adjoint sweep and the light-cone sampler.

Paper: Omlin, Raess, Utkin, "Distributed Parallelization of xPU Stencil
Computations in Julia" (arXiv 2211.15716).

Arrays are numpy float64 of shape (nz, ny, nx), C-contiguous, so x is the
fastest index like the paper's column-major (nx, ny, nz) arrays.  Index 0 and
n-1 of every dimension are halo planes; 1..n-2 are the inner points (the
paper's ``@inn``).  With one process and a periodic dimension the inner
points are the unique points of the global grid.

Readings of the paper that this module fixes (the paper is silent on them):
  * the halo update sends plane ol-1 to the lower neighbour's plane n-1 and
    plane n-ol to the upper neighbour's plane 0 (neighbours share ol planes,
    so those are the same global planes), dimensions in order x, y, z, full
    planes (edges and corners become images in every dimension); with one
    periodic process both neighbours are the process itself;
  * the global grid size per dimension is dims*(n-ol) + ol*(1-period);
  * a field one point larger than the grid in a dimension (a staggered face
    field) has overlap ol+1 in that dimension.

Parity pins (tests/test_oracle_pins.py): constant field stays constant
bit-exactly, discrete Fourier modes decay by the closed-form amplification
factor, sum(T/Ci) is conserved, the maximum principle holds, the step equals
a Kronecker-sum sparse-matrix operator on the periodic torus, the halo equals
a brute-force periodic image map, the adjoint passes the dot-product test and
a closed-form Fourier gradient, and the flux form equals the Laplacian form.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_INT3 = ctypes.c_int * 3


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError("oracle library not built: run oracle/build.py (or __graft_entry__.build())")
        lib = ctypes.CDLL(_build.LIB)
        lib.oracle_halo.argtypes = [_D, _I64, _I64, _I64, _INT3, _INT3]
        lib.oracle_step.argtypes = [_D, _D, _D, _I64, _I64, _I64] + [ctypes.c_double] * 5
        lib.oracle_max.argtypes = [_D, _I64]
        lib.oracle_max.restype = ctypes.c_double
        lib.oracle_dt.argtypes = [ctypes.c_double] * 5
        lib.oracle_dt.restype = ctypes.c_double
        lib.oracle_run.argtypes = [_D, _D, _D, _I64, _I64, _I64, _INT3, _INT3] + \
            [ctypes.c_double] * 5 + [ctypes.c_int]
        lib.oracle_adjoint_step.argtypes = [_D, _D, _D, _D, _D, _I64, _I64, _I64] + [ctypes.c_double] * 5
        lib.oracle_flux.argtypes = [_D, _D, _D, _D, _I64, _I64, _I64] + [ctypes.c_double] * 4
        lib.oracle_flux_update.argtypes = [_D, _D, _D, _D, _D, _D, _I64, _I64, _I64] + [ctypes.c_double] * 4
        lib.oracle_flux_adjoint_step.argtypes = [_D] * 10 + [_I64, _I64, _I64] + [ctypes.c_double] * 5
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _LIB = lib
    return _LIB


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(_D)


def _dims(a):
    nz, ny, nx = a.shape
    return nx, ny, nz


def num_threads():
    return _lib().oracle_num_threads()


def set_num_threads(n):
    _lib().oracle_set_num_threads(int(n))


# --------------------------------------------------------------------------- grid
def global_size(n, dims=(1, 1, 1), periods=(1, 1, 1), overlaps=(2, 2, 2)):
    """Implicit global grid size per dimension (Sec. 2): neighbouring local
    grids share `ol` planes, and a non-periodic edge keeps its `ol` planes."""
    return tuple(int(d) * (int(m) - int(o)) + int(o) * (1 - int(p))
                 for m, d, p, o in zip(n, dims, periods, overlaps))


def field_overlaps(field_shape_xyz, grid_n_xyz, overlaps=(2, 2, 2)):
    """Overlap of one field: a field with one more point than the grid in a
    dimension (staggered faces) overlaps by one more plane."""
    return tuple(int(o) + (int(s) - int(n)) for s, n, o in zip(field_shape_xyz, grid_n_xyz, overlaps))


# --------------------------------------------------------------------------- halo
def halo(A, ol=(2, 2, 2), periods=(1, 1, 1)):
    """In-place halo update of one field (Fig. 1 `update_halo!`); `ol` is this
    field's own overlap per dimension (x, y, z)."""
    nx, ny, nz = _dims(A)
    _lib().oracle_halo(_p(A), nx, ny, nz, _INT3(*ol), _INT3(*periods))
    return A


# --------------------------------------------------------------------------- forward
def max_all(A):
    """maximum(Ci) of Fig. 1 over every point of the array."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    return _lib().oracle_max(_p(A), A.size)


def time_step(dx, dy, dz, lam, max_ci):
    """dt = min(dx^2, dy^2, dz^2)/lam/maximum(Ci)/6.1 (Fig. 1)."""
    return _lib().oracle_dt(dx, dy, dz, lam, max_ci)


def step(T, Ci, lam, dt, dx, dy, dz, out=None):
    """One `step!` of Fig. 1 on the inner points.  Halo points of `out` keep
    whatever they held (a copy of T when `out` is not given)."""
    if out is None:
        out = T.copy()
    nx, ny, nz = _dims(T)
    _lib().oracle_step(_p(out), _p(T), _p(Ci), nx, ny, nz, lam, dt, dx, dy, dz)
    return out


def run(T0, Ci, nt, lam, dt, dx, dy, dz, ol=(2, 2, 2), periods=(1, 1, 1)):
    """nt steps of the Fig. 1 time loop (step, halo update, swap) from T0;
    returns the final state (T0 is not modified)."""
    T = np.array(T0, dtype=np.float64, order="C", copy=True)
    W = np.empty_like(T)
    nx, ny, nz = _dims(T)
    _lib().oracle_run(_p(T), _p(W), _p(Ci), nx, ny, nz, _INT3(*ol), _INT3(*periods),
                      lam, dt, dx, dy, dz, int(nt))
    return T


def run_states(T0, Ci, nt, lam, dt, dx, dy, dz, ol=(2, 2, 2), periods=(1, 1, 1)):
    """Every state T_0..T_nt of the time loop (for small grids)."""
    states = [np.array(T0, dtype=np.float64, copy=True)]
    for _ in range(nt):
        T2 = step(states[-1], Ci, lam, dt, dx, dy, dz, out=states[-1].copy())
        halo(T2, ol, periods)
        states.append(T2)
    return states


# --------------------------------------------------------------------------- light cone
def _periodic_box(A, centre, radius):
    """Gather the (2r+1)^3 box of padded indices centre-r..centre+r from a
    fully periodic, halo-consistent field via the unique-point image map:
    padded index p <-> unique index (p-1) mod N with N = n-2."""
    nz, ny, nx = A.shape
    idx = []
    for c, n in zip(centre[::-1], (nz, ny, nx)):
        N = n - 2
        idx.append((np.arange(c - radius, c + radius + 1) - 1) % N + 1)
    return A[np.ix_(idx[0], idx[1], idx[2])].copy()


def run_points(T0, Ci, nt, lam, dt, dx, dy, dz, points):
    """T_nt at selected inner points (i, j, k) of a fully periodic grid.

    After s steps a point depends only on the initial state within s points of
    it in each dimension, so each sample runs the plain step on the box of
    radius nt around it (gathered through the periodic image map); the box
    boundary is left fixed, and its error travels one point per step inwards,
    reaching the centre only after nt+1 steps.  Returns an array of values."""
    out = []
    zero = (0, 0, 0)
    for (i, j, k) in points:
        Tb = _periodic_box(T0, (i, j, k), nt)
        Cb = _periodic_box(Ci, (i, j, k), nt)
        Tr = run(Tb, Cb, nt, lam, dt, dx, dy, dz, ol=(2, 2, 2), periods=zero)
        out.append(Tr[nt, nt, nt])
    return np.array(out)


# --------------------------------------------------------------------------- adjoint
def adjoint_step(lp, Tn, Ci, gCi, lam, dt, dx, dy, dz, out=None):
    """Transposed step: returns lam_n and accumulates gCi in place (inner
    points).  `lp` and `Ci` must carry valid halos."""
    if out is None:
        out = np.zeros_like(lp)
    nx, ny, nz = _dims(lp)
    _lib().oracle_adjoint_step(_p(out), _p(lp), _p(Tn), _p(Ci), _p(gCi), nx, ny, nz, lam, dt, dx, dy, dz)
    return out


def inner(A):
    return A[1:-1, 1:-1, 1:-1]


def loss(T, T_obs):
    """0.5 * sum over unique points of (T - T_obs)^2, summed exactly rounded."""
    d = (inner(T) - inner(T_obs)).ravel()
    return 0.5 * math.fsum(d * d)


def gradient(T0, Ci, T_obs, nt, lam, dt, dx, dy, dz, every=1, ol=(2, 2, 2), periods=(1, 1, 1)):
    """Loss 0.5*||T_nt - T_obs||^2 over unique points and its gradients with
    respect to the inner points of T0 and Ci, by the adjoint sweep.

    The forward states are recomputed from snapshots taken every `every`
    steps (every=1 keeps all states).  dt is held fixed, not recomputed from
    Ci.  Returns (loss, dL/dT0, dL/dCi) with zero halos in the gradients."""
    # Buffers are made once and reused (a step writes every inner point and
    # the halo update every periodic halo plane; the halo planes of
    # non-periodic dimensions are T0's in every state and zero in lambda),
    # so large grids do not pay for a fresh array per step.
    snaps = {}
    T = np.array(T0, dtype=np.float64, copy=True)
    W = T.copy()
    for it in range(nt):
        if it % every == 0:
            snaps[it] = T.copy()
        step(T, Ci, lam, dt, dx, dy, dz, out=W)
        halo(W, ol, periods)
        T, W = W, T
    L = loss(T, T_obs)
    lp = np.zeros_like(T)
    inner(lp)[...] = inner(T) - inner(T_obs)
    halo(lp, ol, periods)
    ln = np.zeros_like(T)
    gCi = np.zeros_like(T)
    seg = [W] + [T0.copy() for _ in range(min(every, nt) - 2)] if every > 1 else []
    seg_start = ((nt - 1) // every) * every
    while seg_start >= 0:
        seg_end = min(seg_start + every, nt)
        states = [snaps[seg_start]]
        for q in range(seg_end - seg_start - 1):
            states.append(step(states[-1], Ci, lam, dt, dx, dy, dz, out=seg[q]))
            halo(states[-1], ol, periods)
        for it in range(seg_end - 1, seg_start - 1, -1):
            adjoint_step(lp, states[it - seg_start], Ci, gCi, lam, dt, dx, dy, dz, out=ln)
            halo(ln, ol, periods)
            lp, ln = ln, lp
        seg_start -= every
    gT0 = np.zeros_like(T)
    inner(gT0)[...] = inner(lp)
    g = np.zeros_like(T)
    inner(g)[...] = inner(gCi)
    return L, gT0, g


# --------------------------------------------------------------------------- flux form
def face_shapes(T):
    nz, ny, nx = T.shape
    return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)


def flux(T, lam, dx, dy, dz, out=None):
    """Face fluxes q = -lam*grad(T) on faces 1..n-1 of the inner rows."""
    if out is None:
        out = tuple(np.zeros(s) for s in face_shapes(T))
    qx, qy, qz = out
    nx, ny, nz = _dims(T)
    _lib().oracle_flux(_p(qx), _p(qy), _p(qz), _p(T), nx, ny, nz, lam, dx, dy, dz)
    return qx, qy, qz


def flux_update(T, Ci, q, dt, dx, dy, dz, out=None):
    """T2 = T - dt*Ci*div(q) on the inner cells."""
    if out is None:
        out = T.copy()
    nx, ny, nz = _dims(T)
    _lib().oracle_flux_update(_p(out), _p(T), _p(Ci), _p(q[0]), _p(q[1]), _p(q[2]),
                              nx, ny, nz, dt, dx, dy, dz)
    return out


def flux_halo(T, q, overlaps=(2, 2, 2), periods=(1, 1, 1)):
    """Halo update of the cell field and the three face fields."""
    nz, ny, nx = T.shape
    halo(T, overlaps, periods)
    for A in q:
        halo(A, field_overlaps(_dims(A), (nx, ny, nz), overlaps), periods)


def flux_run(T0, Ci, nt, lam, dt, dx, dy, dz, overlaps=(2, 2, 2), periods=(1, 1, 1), return_q=False):
    """nt flux-form steps: fluxes, cell update, halo update of T2, qx, qy, qz."""
    T = np.array(T0, dtype=np.float64, copy=True)
    q = tuple(np.zeros(s) for s in face_shapes(T))
    for _ in range(nt):
        flux(T, lam, dx, dy, dz, out=q)
        T2 = flux_update(T, Ci, q, dt, dx, dy, dz, out=T.copy())
        flux_halo(T2, q, overlaps, periods)
        T = T2
    return (T, q) if return_q else T


def flux_run_points(T0, Ci, nt, lam, dt, dx, dy, dz, points):
    """T_nt of the flux-form time loop at selected inner cells (i, j, k) of a
    fully periodic grid, by the light-cone argument of run_points: a cell's
    faces and update read only its six neighbours, so after s steps a cell
    depends on the cells within s of it, and each sample runs flux_run on the
    box of radius nt around it with the box boundary held fixed."""
    out = []
    zero = (0, 0, 0)
    for (i, j, k) in points:
        Tb = _periodic_box(T0, (i, j, k), nt)
        Cb = _periodic_box(Ci, (i, j, k), nt)
        Tr = flux_run(Tb, Cb, nt, lam, dt, dx, dy, dz, overlaps=(2, 2, 2), periods=zero)
        out.append(Tr[nt, nt, nt])
    return np.array(out)


def flux_adjoint_step(lp, Ci, q, gCi, lam, dt, dx, dy, dz, out=None):
    """Transposed flux-form step; q are the forward fluxes of step n."""
    if out is None:
        out = np.zeros_like(lp)
    pm = tuple(np.zeros(s) for s in face_shapes(lp))
    nx, ny, nz = _dims(lp)
    _lib().oracle_flux_adjoint_step(_p(out), _p(lp), _p(Ci), _p(q[0]), _p(q[1]), _p(q[2]),
                                    _p(pm[0]), _p(pm[1]), _p(pm[2]), _p(gCi),
                                    nx, ny, nz, lam, dt, dx, dy, dz)
    return out


def flux_gradient(T0, Ci, T_obs, nt, lam, dt, dx, dy, dz, ol=(2, 2, 2), periods=(1, 1, 1)):
    """Loss and gradients of the flux-form time loop (all states kept)."""
    states = [np.array(T0, dtype=np.float64, copy=True)]
    fluxes = []
    for _ in range(nt):
        T = states[-1]
        q = flux(T, lam, dx, dy, dz)
        T2 = flux_update(T, Ci, q, dt, dx, dy, dz, out=T.copy())
        flux_halo(T2, q, ol, periods)
        states.append(T2)
        fluxes.append(q)
    L = loss(states[-1], T_obs)
    lp = np.zeros_like(T0)
    inner(lp)[...] = inner(states[-1]) - inner(T_obs)
    halo(lp, ol, periods)
    gCi = np.zeros_like(T0)
    for it in range(nt - 1, -1, -1):
        ln = flux_adjoint_step(lp, Ci, fluxes[it], gCi, lam, dt, dx, dy, dz)
        halo(ln, ol, periods)
        lp = ln
    gT0 = np.zeros_like(T0)
    inner(gT0)[...] = inner(lp)
    g = np.zeros_like(T0)
    inner(g)[...] = inner(gCi)
    return L, gT0, g


# --------------------------------------------------------------------------- metrics
def unique_sum(A):
    """Exactly rounded sum over the inner (unique) points."""
    return math.fsum(inner(A).ravel())


def rel_max_err(a, b):
    """max|a-b| / max|b| over the inner (unique) points."""
    a = inner(np.asarray(a, dtype=np.float64))
    b = inner(np.asarray(b, dtype=np.float64))
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
