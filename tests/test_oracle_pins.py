"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's formulas: each checks it against an
independent statement -- the paper's own worked example (Fig. 1 listing),
a closed form, an invariant, a different formulation of the same operator
(sparse Kronecker-sum matrices on the periodic torus of unique points,
dense Jacobian products), a brute-force index map, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2211_15716_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PER = (1, 1, 1)


def _inner(A):
    return A[1:-1, 1:-1, 1:-1]


def _periodic_d2(N):
    """1-D periodic second-difference matrix on N unique points (wrap by
    modular indexing, so N=1 gives 0 and N=2 gives [[-2,2],[2,-2]])."""
    D = np.zeros((N, N))
    for u in range(N):
        D[u, (u + 1) % N] += 1.0
        D[u, (u - 1) % N] += 1.0
        D[u, u] -= 2.0
    return D


def _kron_laplacian(nx, ny, nz, dx, dy, dz):
    """Kronecker-sum Laplacian on the unique points (x fastest)."""
    Nx, Ny, Nz = nx - 2, ny - 2, nz - 2
    Ix, Iy, Iz = sp.identity(Nx), sp.identity(Ny), sp.identity(Nz)
    Dx, Dy, Dz = (sp.csr_matrix(_periodic_d2(N)) for N in (Nx, Ny, Nz))
    return (sp.kron(sp.kron(Iz, Iy), Dx) / dx**2 + sp.kron(sp.kron(Iz, Dy), Ix) / dy**2 +
            sp.kron(sp.kron(Dz, Iy), Ix) / dz**2).tocsr()


def _with_halo(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    oracle.halo(A, (2, 2, 2), PER)
    return A


# --------------------------------------------------------------------------- the paper's example
def test_fig1_listing_constant_state_is_exact():
    """Fig. 1 runs from T = 1.7, Ci = 1/c0: every step must leave T unchanged
    bit for bit (second differences of a constant are exactly zero)."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_listing.json")))
    n = 24  # same recipe as the listing, smaller edge so the suite stays fast
    n_g = oracle.global_size((g["nx"],) * 3, periods=(0, 0, 0))
    assert n_g == (g["expected_global_size"],) * 3
    dx = g["lx"] / (n_g[0] - 1)
    assert dx == 1.0 / 511
    Ci = np.full((n, n, n), 1.0 / g["c0"])
    dt = oracle.time_step(dx, dx, dx, g["lam"], oracle.max_all(Ci))
    assert dt == (1.0 / 511) ** 2 / 1.0 / 0.5 / 6.1
    T0 = np.full((n, n, n), g["T_init"])
    for periods in ((0, 0, 0), (1, 1, 1)):
        T = oracle.run(T0, Ci, g["nt"], g["lam"], dt, dx, dx, dx, periods=periods)
        assert np.array_equal(T, T0)


# --------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("m", [(1, 0, 0), (1, 2, 3), (2, 1, 1), "checker"])
def test_fourier_mode_decays_by_closed_form(m):
    """A single discrete Fourier mode with constant Ci is an eigenvector of
    the periodic step: amplitude B*G^nt with
    G = 1 - dt*lam*Ci*sum_d 4/dd^2 sin^2(pi m_d / N_d)."""
    nx, ny, nz = 14, 10, 12
    if m == "checker":
        m = ((nx - 2) // 2, (ny - 2) // 2, (nz - 2) // 2)
    dx, dy, dz = 1.0 / 13, 1.3 / 9, 0.8 / 11
    lam, c, A, B, nt = 1.0, 0.5, 1.7, 0.1, 12
    T0 = synth.fourier_mode(nx, ny, nz, m, A, B)
    Ci = np.full_like(T0, c)
    dt = oracle.time_step(dx, dy, dz, lam, c)
    G = 1.0 - dt * lam * c * sum(4.0 / d**2 * math.sin(math.pi * md / (n - 2)) ** 2
                                 for md, n, d in zip(m, (nx, ny, nz), (dx, dy, dz)))
    T = oracle.run(T0, Ci, nt, lam, dt, dx, dy, dz)
    phi = (T0 - A) / B
    expect = A + B * G**nt * phi
    assert np.max(np.abs(T - expect)) <= 1e-12 * B
    if m == ((nx - 2) // 2, (ny - 2) // 2, (nz - 2) // 2) and dx == dy == dz:
        assert abs(G - (1 - 12 / 6.1)) < 1e-15


def test_step_equals_kronecker_sum_operator():
    """T1 = T + dt*lam*Ci .* (L T) with L the Kronecker-sum periodic
    Laplacian on the unique points, anisotropic sizes and spacings."""
    nx, ny, nz = 9, 7, 6
    dx, dy, dz = 0.11, 0.13, 0.17
    lam = 0.9
    T, Ci = synth.uniform_fields(nx, ny, nz, seed=3, lo=0.2, hi=1.0, n=2)
    T, Ci = _with_halo(T), _with_halo(Ci)
    dt = oracle.time_step(dx, dy, dz, lam, oracle.max_all(Ci))
    L = _kron_laplacian(nx, ny, nz, dx, dy, dz)
    t = _inner(T).ravel()
    expect = t + dt * lam * _inner(Ci).ravel() * (L @ t)
    T1 = oracle.step(T, Ci, lam, dt, dx, dy, dz)
    oracle.halo(T1)
    assert np.max(np.abs(_inner(T1).ravel() - expect)) <= 1e-14 * np.max(np.abs(expect))
    # and the halo of the result is the periodic image of its inner points
    assert np.array_equal(T1, _with_halo(T1.copy()))


def test_textbook_1d_ftcs_line():
    """A field varying only in x reduces each (j,k) line to the 1-D FTCS heat
    update, here as a dense matrix product on the line's unique points."""
    nx, ny, nz = 12, 5, 6
    dx = dy = dz = 1.0 / 11
    rng = np.random.default_rng(7)
    line = rng.uniform(1.0, 2.0, nx)
    T = np.broadcast_to(line, (nz, ny, nx)).copy()
    Ci = np.broadcast_to(rng.uniform(0.25, 0.75, nx), (nz, ny, nx)).copy()
    T, Ci = _with_halo(T), _with_halo(Ci)
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    nt = 5
    D = _periodic_d2(nx - 2)
    M = np.eye(nx - 2) + dt * np.diag(Ci[0, 0, 1:-1]) @ D / dx**2
    expect = np.linalg.matrix_power(M, nt) @ T[0, 0, 1:-1]
    Tn = oracle.run(T, Ci, nt, 1.0, dt, dx, dy, dz)
    for k in range(1, nz - 1):
        for j in range(1, ny - 1):
            assert np.max(np.abs(Tn[k, j, 1:-1] - expect)) <= 1e-14 * np.max(expect)


def test_degenerate_single_unique_point():
    """n = 3 per dimension leaves one unique point: every neighbour is its
    own image, so the step changes nothing."""
    T, Ci = synth.uniform_fields(3, 3, 3, seed=1, lo=0.5, hi=1.5, n=2)
    T, Ci = _with_halo(T), _with_halo(Ci)
    assert np.all(T == T[1, 1, 1])
    Tn = oracle.run(T, Ci, 4, 1.0, 1e-3, 0.5, 0.5, 0.5)
    assert np.array_equal(Tn, T)


# --------------------------------------------------------------------------- invariants
def test_conservation_of_T_over_Ci():
    """sum(T/Ci) over unique points is conserved for any positive Ci, and
    sum(T) for constant Ci (the periodic Laplacian sums to zero)."""
    nx, ny, nz = 16, 13, 11
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=2, noise=1e-2)
    T0, Ci = _with_halo(T0), _with_halo(Ci)
    dx = dy = dz = 1.0 / 15
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    T = oracle.run(T0, Ci, 20, 1.0, dt, dx, dy, dz)
    s0 = math.fsum((_inner(T0) / _inner(Ci)).ravel())
    s1 = math.fsum((_inner(T) / _inner(Ci)).ravel())
    assert abs(s1 - s0) <= 1e-12 * abs(s0)
    Cc = np.full_like(Ci, 0.4)
    T = oracle.run(T0, Cc, 20, 1.0, dt, dx, dy, dz)
    assert abs(oracle.unique_sum(T) - oracle.unique_sum(T0)) <= 1e-12 * abs(oracle.unique_sum(T0))


def test_maximum_principle():
    """The centre weight 1 - 6*Ci/(6.1*max Ci) is positive: each step is a
    convex combination, so min never decreases and max never increases."""
    n = 14
    T, Ci = synth.noisy_state_uniform_ci(n, n, n, seed=4, noise=0.05)
    T, Ci = _with_halo(T), _with_halo(Ci)
    dx = 1.0 / (n - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    lo, hi = _inner(T).min(), _inner(T).max()
    for _ in range(15):
        T = oracle.run(T, Ci, 1, 1.0, dt, dx, dx, dx)
        assert _inner(T).min() >= lo - 4e-16 * abs(lo)
        assert _inner(T).max() <= hi + 4e-16 * abs(hi)
        lo, hi = _inner(T).min(), _inner(T).max()


# --------------------------------------------------------------------------- halo and grid
def _image(n, ol):
    """Periodic image map of one dimension after the halo update: the first
    plane takes plane n-ol, the last plane takes plane ol-1."""
    img = np.arange(n)
    img[0] = n - ol
    img[n - 1] = ol - 1
    return img


@pytest.mark.parametrize("shape,ol,periods", [
    ((3, 3, 3), (2, 2, 2), (1, 1, 1)),
    ((4, 5, 6), (2, 2, 2), (1, 1, 1)),
    ((7, 3, 5), (2, 2, 2), (1, 0, 1)),
    ((33, 17, 9), (2, 2, 2), (0, 1, 1)),
    ((13, 12, 12), (3, 2, 2), (1, 1, 1)),   # staggered x-face field of a 12^3 grid
    ((12, 13, 12), (2, 3, 2), (1, 1, 1)),
    ((12, 12, 13), (2, 2, 3), (1, 1, 0)),
    ((10, 11, 12), (4, 3, 2), (1, 1, 1)),   # wider overlaps
])
def test_halo_equals_bruteforce_image(shape, ol, periods):
    nx, ny, nz = shape
    A = synth.uniform_fields(nx, ny, nz, seed=11, n=1)[0]
    ref = A.copy()
    imgs = [(_image(n, o) if p else np.arange(n)) for n, o, p in zip(shape, ol, periods)]
    expect = ref[np.ix_(imgs[2], imgs[1], imgs[0])]
    oracle.halo(A, ol, periods)
    assert np.array_equal(A, expect)


def test_global_size_is_union_of_overlapping_local_grids():
    """Neighbouring local grids share `ol` planes; a periodic dimension also
    shares them across the wrap.  Count the union of index sets directly."""
    for n, P, ol in [(512, 1, 2), (10, 2, 2), (10, 3, 4), (7, 5, 2)]:
        for per in (0, 1):
            pts = set()
            for r in range(P):
                for i in range(n):
                    pts.add(r * (n - ol) + i)
            size = len(pts)
            if per:  # the last `ol` planes coincide with the first ones
                size -= ol
            assert oracle.global_size((n, n, n), (P, P, P), (per,) * 3, (ol,) * 3) == (size,) * 3


# --------------------------------------------------------------------------- adjoint
def _dense_step_matrix(Ci, lam, dt, dx, dy, dz):
    nz, ny, nx = Ci.shape
    L = _kron_laplacian(nx, ny, nz, dx, dy, dz).toarray()
    return np.eye(L.shape[0]) + dt * lam * np.diag(_inner(Ci).ravel()) @ L


def test_adjoint_equals_dense_jacobian_transpose():
    """dL/dT0 from the adjoint sweep equals J^T r with J the product of dense
    step matrices and r = T_nt - T_obs (no adjoint code involved in J)."""
    nx, ny, nz = 7, 6, 8
    dx, dy, dz = 0.2, 0.25, 0.15
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=5, lo=0.3, hi=1.0, n=3)
    T0, Ci, Tobs = _with_halo(T0), _with_halo(Ci), _with_halo(Tobs)
    lam, nt = 1.0, 6
    dt = oracle.time_step(dx, dy, dz, lam, oracle.max_all(Ci))
    L, gT0, gCi = oracle.gradient(T0, Ci, Tobs, nt, lam, dt, dx, dy, dz)
    M = _dense_step_matrix(Ci, lam, dt, dx, dy, dz)
    J = np.linalg.matrix_power(M, nt)
    r = J @ _inner(T0).ravel() - _inner(Tobs).ravel()
    assert abs(L - 0.5 * float(r @ r)) <= 1e-13 * L
    expect = J.T @ r
    assert np.max(np.abs(_inner(gT0).ravel() - expect)) <= 1e-13 * np.max(np.abs(expect))


def test_adjoint_dot_product():
    """<J d, y> = <d, J^T y> for the linear map T0 -> T_nt."""
    nx, ny, nz = 10, 9, 8
    dx = dy = dz = 1.0 / 9
    d, Ci, y = synth.uniform_fields(nx, ny, nz, seed=6, lo=0.2, hi=1.0, n=3)
    d, Ci, y = _with_halo(d), _with_halo(Ci), _with_halo(y)
    nt = 9
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    Jd = oracle.run(d, Ci, nt, 1.0, dt, dx, dy, dz)
    Tobs = Jd - y  # so that the adjoint's residual is exactly y on unique points
    _, JTy, _ = oracle.gradient(d, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    lhs = math.fsum((_inner(Jd) * _inner(Jd - Tobs)).ravel())
    rhs = math.fsum((_inner(d) * _inner(JTy)).ravel())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_ci_gradient_matches_central_differences():
    nx, ny, nz = 6, 7, 5
    dx, dy, dz = 0.2, 0.17, 0.25
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=8, lo=0.3, hi=0.9, n=3)
    T0, Ci, Tobs = _with_halo(T0), _with_halo(Ci), _with_halo(Tobs)
    nt = 7
    dt = oracle.time_step(dx, dy, dz, 1.0, 1.0)  # fixed, not recomputed from Ci
    _, _, gCi = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    g = _inner(gCi)
    for (k, j, i) in [(1, 1, 1), (2, 3, 1), (3, 5, 4), (1, 2, 3)]:
        h = 1e-4 * Ci[k, j, i]
        vals = []
        for s in (+1, -1):
            C2 = Ci.copy()
            C2[k, j, i] += s * h
            oracle.halo(C2)  # the perturbed unique point moves its images too
            vals.append(oracle.loss(oracle.run(T0, C2, nt, 1.0, dt, dx, dy, dz), Tobs))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k - 1, j - 1, i - 1]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(g)))


def test_ci_gradient_fourier_closed_form():
    """Uniform Ci = c, T0 = A + B*phi: T_nt = A + B*G(c)^nt*phi, so the sum of
    dL/dCi over all unique points is sum r*B*nt*G^(nt-1)*dG/dc*phi."""
    nx, ny, nz = 10, 12, 8
    dx, dy, dz = 0.1, 0.09, 0.13
    m, A, B, c, nt = (1, 2, 1), 1.7, 0.2, 0.5, 10
    T0 = synth.fourier_mode(nx, ny, nz, m, A, B)
    Tobs = _with_halo(synth.uniform_fields(nx, ny, nz, seed=9, lo=1.5, hi=1.9, n=1)[0])
    Ci = np.full_like(T0, c)
    dt = oracle.time_step(dx, dy, dz, 1.0, 0.6)
    lam_m = -sum(4.0 / d**2 * math.sin(math.pi * md / (n - 2)) ** 2
                 for md, n, d in zip(m, (nx, ny, nz), (dx, dy, dz)))
    G = 1.0 + dt * c * lam_m
    phi = _inner((T0 - A) / B)
    r = A + B * G**nt * phi - _inner(Tobs)
    expect = math.fsum((r * B * nt * G ** (nt - 1) * dt * lam_m * phi).ravel())
    _, _, gCi = oracle.gradient(T0, Ci, Tobs, nt, 1.0, dt, dx, dy, dz)
    got = math.fsum(_inner(gCi).ravel())
    assert abs(got - expect) <= 1e-12 * abs(expect)


def test_checkpointed_gradient_equals_store_all():
    nx = ny = nz = 9
    dx = 1.0 / 8
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=10, lo=0.3, hi=0.9, n=3)
    T0, Ci, Tobs = _with_halo(T0), _with_halo(Ci), _with_halo(Tobs)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    ref = oracle.gradient(T0, Ci, Tobs, 11, 1.0, dt, dx, dx, dx, every=1)
    for every in (3, 4, 11, 16):
        got = oracle.gradient(T0, Ci, Tobs, 11, 1.0, dt, dx, dx, dx, every=every)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


# --------------------------------------------------------------------------- flux form
def test_flux_form_equals_laplacian_form():
    nx, ny, nz = 11, 9, 10
    dx, dy, dz = 0.1, 0.12, 0.11
    T0, Ci = synth.noisy_state_uniform_ci(nx, ny, nz, seed=12, noise=1e-2)
    T0, Ci = _with_halo(T0), _with_halo(Ci)
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    a = oracle.run(T0, Ci, 8, 1.0, dt, dx, dy, dz)
    b, q = oracle.flux_run(T0, Ci, 8, 1.0, dt, dx, dy, dz, return_q=True)
    assert oracle.rel_max_err(b, a) <= 1e-13
    # after the halo update every face field is periodic: face f and face f+N agree
    qx, qy, qz = q
    assert np.array_equal(qx[:, :, nx - 1], qx[:, :, 1]) and np.array_equal(qx[:, :, 0], qx[:, :, nx - 2])
    assert np.array_equal(qy[:, ny - 1, :], qy[:, 1, :]) and np.array_equal(qz[nz, :, :], qz[2, :, :])


def test_flux_gradient_equals_laplacian_gradient():
    nx, ny, nz = 7, 8, 6
    dx, dy, dz = 0.2, 0.18, 0.22
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=13, lo=0.3, hi=0.9, n=3)
    T0, Ci, Tobs = _with_halo(T0), _with_halo(Ci), _with_halo(Tobs)
    dt = oracle.time_step(dx, dy, dz, 1.0, oracle.max_all(Ci))
    a = oracle.gradient(T0, Ci, Tobs, 6, 1.0, dt, dx, dy, dz)
    b = oracle.flux_gradient(T0, Ci, Tobs, 6, 1.0, dt, dx, dy, dz)
    assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0])
    for x, y in ((a[1], b[1]), (a[2], b[2])):
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(x))


def test_light_cone_sampler_matches_full_run():
    n, nt = 20, 6
    T0, Ci = synth.noisy_state_uniform_ci(n, n, n, seed=14, noise=1e-2)
    T0, Ci = _with_halo(T0), _with_halo(Ci)
    dx = 1.0 / (n - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    full = oracle.run(T0, Ci, nt, 1.0, dt, dx, dx, dx)
    pts = [(1, 1, 1), (18, 18, 18), (5, 11, 17), (10, 2, 9)]
    got = oracle.run_points(T0, Ci, nt, 1.0, dt, dx, dx, dx, pts)
    assert np.array_equal(got, np.array([full[k, j, i] for (i, j, k) in pts]))


# --------------------------------------------------------------------------- adjoint with non-periodic dimensions
def _d2_line(N, periodic):
    """1-D second difference on the N unknowns of a line: with a periodic
    wrap, or with the line's two outer neighbours fixed boundary values (they
    only add a constant, so the matrix couples the unknowns alone)."""
    if periodic:
        return _periodic_d2(N)
    D = -2.0 * np.eye(N)
    D += np.eye(N, k=1) + np.eye(N, k=-1)
    return D


def _affine_operator(T0, periods, spacings):
    """The step on the inner points of a grid whose non-periodic dimensions
    keep their boundary planes fixed, as t -> t + a*c.*(L t + b): L is the
    Kronecker sum of the per-dimension line operators (x fastest) and b the
    fixed boundary planes' contribution, read straight from T0."""
    nz, ny, nx = T0.shape
    Ns = (nx - 2, ny - 2, nz - 2)
    I = [np.eye(N) for N in Ns]
    D = [_d2_line(N, p) / d**2 for N, p, d in zip(Ns, periods, spacings)]
    L = (np.kron(np.kron(I[2], I[1]), D[0]) + np.kron(np.kron(I[2], D[1]), I[0]) +
         np.kron(np.kron(D[2], I[1]), I[0]))
    b = np.zeros((nz - 2, ny - 2, nx - 2))
    dx, dy, dz = spacings
    if not periods[0]:
        b[:, :, 0] += T0[1:-1, 1:-1, 0] / dx**2
        b[:, :, -1] += T0[1:-1, 1:-1, -1] / dx**2
    if not periods[1]:
        b[:, 0, :] += T0[1:-1, 0, 1:-1] / dy**2
        b[:, -1, :] += T0[1:-1, -1, 1:-1] / dy**2
    if not periods[2]:
        b[0, :, :] += T0[0, 1:-1, 1:-1] / dz**2
        b[-1, :, :] += T0[-1, 1:-1, 1:-1] / dz**2
    return L, b.ravel()


@pytest.mark.parametrize("periods", [(1, 0, 1), (0, 0, 0), (0, 1, 1)])
def test_gradient_with_fixed_boundary_planes_equals_dense_formulation(periods):
    """In a non-periodic dimension the boundary planes are fixed inputs: the
    unknowns are the inner points, each step is the affine map
    t -> t + a*c.*(L t + b), the loss 0.5*|t_nt - t_obs|^2 over them.  Its
    gradients follow from dense matrices with no adjoint code involved:
      dL/dT0 = (M^nt)^T r,  M = I + a*diag(c)*L,  r = t_nt - t_obs,
      dL/dCi = sum_n a*lam_{n+1} .* (L t_n + b),  lam_{n+1} = (M^T)^(nt-1-n) r.
    The oracle's forward run, loss and both gradients must agree (so lambda
    carries nothing into the boundary planes), and central differences
    confirm the Ci gradient at points next to a fixed boundary."""
    nx, ny, nz = 7, 6, 8
    spacings = (0.19, 0.23, 0.16)
    T0, Ci, Tobs = synth.uniform_fields(nx, ny, nz, seed=41, lo=0.3, hi=1.0, n=3)
    for A in (T0, Ci, Tobs):
        oracle.halo(A, (2, 2, 2), periods)
    lam, nt = 0.8, 7
    dt = oracle.time_step(*spacings, lam, oracle.max_all(Ci))
    a = dt * lam
    L, b = _affine_operator(T0, periods, spacings)
    c = _inner(Ci).ravel()
    M = np.eye(L.shape[0]) + a * np.diag(c) @ L
    ts = [_inner(T0).ravel().copy()]
    for _ in range(nt):
        t = ts[-1]
        ts.append(t + a * c * (L @ t + b))
    T_nt = oracle.run(T0, Ci, nt, lam, dt, *spacings, periods=periods)
    assert np.max(np.abs(_inner(T_nt).ravel() - ts[-1])) <= 1e-13 * np.max(np.abs(ts[-1]))
    r = ts[-1] - _inner(Tobs).ravel()
    gT_expect = np.linalg.matrix_power(M, nt).T @ r
    gC_expect = np.zeros_like(c)
    lam_v = r.copy()
    for n in range(nt - 1, -1, -1):
        gC_expect += a * lam_v * (L @ ts[n] + b)
        lam_v = M.T @ lam_v
    Lval, gT0, gCi = oracle.gradient(T0, Ci, Tobs, nt, lam, dt, *spacings, periods=periods)
    assert abs(Lval - 0.5 * float(r @ r)) <= 1e-13 * Lval
    assert np.max(np.abs(_inner(gT0).ravel() - gT_expect)) <= 1e-12 * np.max(np.abs(gT_expect))
    assert np.max(np.abs(_inner(gCi).ravel() - gC_expect)) <= 1e-12 * np.max(np.abs(gC_expect))
    # boundary planes carry no gradient
    for G in (gT0, gCi):
        assert np.all(G[0] == 0) and np.all(G[-1] == 0) and np.all(G[:, 0] == 0) and np.all(G[:, :, -1] == 0)
    # central differences in Ci next to the fixed boundary (and inside)
    g = _inner(gCi)
    for (k, j, i) in [(1, 1, 1), (nz - 2, ny - 2, nx - 2), (3, 1, 5), (1, 4, 3)]:
        h = 1e-4 * Ci[k, j, i]
        vals = []
        for s in (+1, -1):
            C2 = Ci.copy()
            C2[k, j, i] += s * h
            oracle.halo(C2, (2, 2, 2), periods)
            vals.append(oracle.loss(oracle.run(T0, C2, nt, lam, dt, *spacings, periods=periods), Tobs))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k - 1, j - 1, i - 1]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(g)))


def test_flux_light_cone_sampler_matches_full_run():
    n, nt = 20, 6
    T0, Ci = synth.noisy_state_uniform_ci(n, n, n, seed=15, noise=1e-2)
    T0, Ci = _with_halo(T0), _with_halo(Ci)
    dx = 1.0 / (n - 1)
    dt = oracle.time_step(dx, dx, dx, 1.0, oracle.max_all(Ci))
    full = oracle.flux_run(T0, Ci, nt, 1.0, dt, dx, dx, dx)
    pts = [(1, 1, 1), (18, 18, 18), (5, 11, 17), (10, 2, 9)]
    got = oracle.flux_run_points(T0, Ci, nt, 1.0, dt, dx, dx, dx, pts)
    assert np.array_equal(got, np.array([full[k, j, i] for (i, j, k) in pts]))
