"""Seeded synthetic inputs for the diffusion workloads.

This module only draws random numbers and evaluates initial conditions on grid
coordinates; it holds none of the method's arithmetic (no halo update, no step,
no time step).  Both the HIP path and the CPU oracle receive its arrays as
data.  The returned fields are raw: their halo planes still hold the values
drawn for them, and each side applies its own halo update before stepping.

Recipes (paper: Fig. 1 heat-diffusion setup, lam = 1, c0 = 2, lx = ly = lz = 1):
  * coordinates x_i = i*dx for local index i = 0..nx-1, dx = lx/(nx-1);
  * "gaussian" state T0 = 1.7 + exp(-((x-.5)^2+(y-.5)^2+(z-.5)^2)/0.01),
    plus 1e-3 * N(0,1) noise when requested;
  * Ci drawn after the noise from the same generator: (1/c0)*U(0.5, 1.5),
    or lognormal exp(log(0.5) + 0.2*N(0,1));
  * arrays are float64 of shape (nz, ny, nx), drawn in x-fastest order from
    numpy.random.default_rng(seed).
"""
import numpy as np

LAM = 1.0
C0 = 2.0
LX = LY = LZ = 1.0


def spacing(n, length=1.0):
    return length / (n - 1)


def coords(n, length=1.0):
    return np.arange(n, dtype=np.float64) * spacing(n, length)


def gaussian_bump(nx, ny, nz, base=1.7, width=0.01):
    x = coords(nx, LX)[None, None, :]
    y = coords(ny, LY)[None, :, None]
    z = coords(nz, LZ)[:, None, None]
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    return base + np.exp(-r2 / width)


def _shape(nx, ny, nz):
    return (nz, ny, nx)


def noisy_state_uniform_ci(nx, ny, nz, seed=0, noise=1e-3, c0=C0):
    """T0 = 1.7 + gaussian bump + noise*N(0,1); Ci = (1/c0)*U(0.5, 1.5)."""
    rng = np.random.default_rng(seed)
    T0 = gaussian_bump(nx, ny, nz)
    if noise:
        T0 += noise * rng.standard_normal(_shape(nx, ny, nz))
    Ci = rng.uniform(0.5, 1.5, _shape(nx, ny, nz)) / c0
    return T0, Ci


def bump_state_lognormal_ci(nx, ny, nz, seed=0, mu=np.log(0.5), sigma=0.2):
    """T0 = 1.7 + gaussian bump (no noise); Ci = exp(mu + sigma*N(0,1))."""
    rng = np.random.default_rng(seed)
    T0 = gaussian_bump(nx, ny, nz)
    Ci = np.exp(mu + sigma * rng.standard_normal(_shape(nx, ny, nz)))
    return T0, Ci


def sine_ci(nx, ny, nz, base=0.5, amp=0.3):
    """Ci_true = base*(1 + amp*sin(2 pi x) sin(2 pi y) sin(2 pi z))."""
    x = coords(nx, LX)[None, None, :]
    y = coords(ny, LY)[None, :, None]
    z = coords(nz, LZ)[:, None, None]
    return base * (1.0 + amp * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z))


def uniform_fields(nx, ny, nz, seed=0, lo=-1.0, hi=1.0, n=1):
    """n independent uniform random fields (for halo and adjoint tests)."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo, hi, _shape(nx, ny, nz)) for _ in range(n)]


def fourier_mode(nx, ny, nz, m=(1, 1, 1), A=1.7, B=0.1):
    """A + B*prod_d cos(2 pi m_d (i_d - 1)/N_d) with N_d = n_d - 2: a single
    discrete Fourier mode on the unique points 1..n-2 of a periodic grid.
    Values on the halo planes are the periodic images."""
    def c(n, md):
        N = n - 2
        i = np.arange(n, dtype=np.float64)
        return np.cos(2 * np.pi * md * (i - 1) / N)
    return A + B * (c(nz, m[2])[:, None, None] * c(ny, m[1])[None, :, None] * c(nx, m[0])[None, None, :])


# --------------------------------------------------------------------------- hashed fields
# Fields too large to draw on the host (billions of points): each point's
# value is offset + u, u = h * 2^-32 in [0, 1), where h is a 32-bit integer
# hash of the point's linear index (x fastest) xor a seed -- two rounds of
# x = ((x >> 16) ^ x) * 0x45d9f3b mod 2^32, then x ^= x >> 16 (Thomas
# Mueller's public-domain integer hash).  Every product stays below 2^59, so
# int64 arithmetic is exact on numpy and torch alike, and the same values
# come out on the device (whole field) and on the host (any chosen points).
_M32 = 0xFFFFFFFF
_HK = 0x45D9F3B


def _hash32(x):
    x = (((x >> 16) ^ x) * _HK) & _M32
    x = (((x >> 16) ^ x) * _HK) & _M32
    return (x >> 16) ^ x


def hashed_uniform(index, seed):
    """u in [0, 1) for linear indices (numpy, each below 2^32)."""
    x = (np.asarray(index, dtype=np.int64) ^ np.int64(seed)) & _M32
    return _hash32(x).astype(np.float64) * 2.0 ** -32


def hashed_field_torch(nx, ny, nz, seed, offset, device, planes=64):
    """offset + u at every point of an (nz, ny, nx) float64 torch tensor on
    `device`, made plane block by plane block (the values equal
    offset + hashed_uniform(i + nx*(j + ny*k), seed))."""
    import torch
    if nx * ny * nz >= 1 << 32:
        raise ValueError("hashed fields index at most 2^32 points")
    out = torch.empty((nz, ny, nx), dtype=torch.float64, device=device)
    plane = nx * ny
    base = torch.arange(plane, dtype=torch.int64, device=device)
    for k0 in range(0, nz, planes):
        k1 = min(nz, k0 + planes)
        ks = torch.arange(k0, k1, dtype=torch.int64, device=device)
        x = ((base[None, :] + ks[:, None] * plane) ^ seed) & _M32
        u = _hash32(x).to(torch.float64) * 2.0 ** -32
        out[k0:k1] = (u + offset).view(k1 - k0, ny, nx)
        del x, u
    return out


# --------------------------------------------------------------------------- named workloads
def workload(name, seed=0, n=None):
    """The named workloads of the diffusion study.

    Returns a dict: T0, Ci (raw float64, no halo applied), nx, ny, nz, lam,
    dx, dy, dz, nt, split and a description.  `n` overrides the cube edge for
    scaled-down variants of the same recipe."""
    if name == "c1_32_fp64":
        n = n or 32
        T0, Ci = noisy_state_uniform_ci(n, n, n, seed)
        nt, split, desc = 10, (16, 2, 2), "32^3 FP64, nt=10, noisy bump, Ci=U(0.5,1.5)/2"
    elif name == "c2_512_fp64":
        n = n or 512
        T0, Ci = bump_state_lognormal_ci(n, n, n, seed)
        nt, split, desc = 100, (16, 2, 2), "512^3 FP64, nt=100, bump, lognormal Ci"
    elif name == "c3_512":
        n = n or 512
        T0, Ci = noisy_state_uniform_ci(n, n, n, seed)
        nt, split, desc = 100, (16, 2, 2), "512^3, nt=100, noisy bump, Ci=U(0.5,1.5)/2"
    elif name == "c4_256_inverse":
        n = n or 256
        T0, _ = noisy_state_uniform_ci(n, n, n, seed)
        Ci = sine_ci(n, n, n)
        nt, split, desc = 200, (16, 2, 2), "256^3 FP64 inverse, nt=200, Ci_true sine"
    elif name == "c5_768_flux":
        n = n or 768
        T0, Ci = noisy_state_uniform_ci(n, n, n, seed)
        nt, split, desc = 100, None, "768^3 FP32 staggered flux form, nt=100"
    else:
        raise KeyError(name)
    nz, ny, nx = T0.shape
    return dict(T0=T0, Ci=Ci, nx=nx, ny=ny, nz=nz, lam=LAM,
                dx=spacing(nx, LX), dy=spacing(ny, LY), dz=spacing(nz, LZ),
                nt=nt, split=split, desc=desc, seed=seed)
