"""Seeded synthetic inputs for the double-diffusive porous-cavity workloads.

This module holds no arithmetic of the lattice Boltzmann method: it only draws the
inputs (initial noise, porosity fields, parameter sweeps, request streams) that both the
GPU library and the CPU oracle are given.  Parameters are plain dictionaries of the
problem statement of the paper (Ra, Pr, Le, Da, N, porosity, ...); each side maps them
to lattice units with its own code.

The paper's cavities (sections 4.1-4.3) are 100x200, 100x100 and 128x128 with a uniform
porosity; the workloads below extend them with synthetic porosity fields and sweeps.
Every draw uses ``numpy.random.default_rng`` with the stated seed.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtr

# Walls of the hot-path cavity: left held at (Th, Ch), right at (Tl, Cl), bottom and top
# adiabatic and impermeable.
CAVITY_SIDES = ("hot", "cold", "adiabatic", "adiabatic")


def noise_fields(nx: int, ny: int, seed, amp: float = 1e-3, T0: float = 0.5, C0: float = 0.5):
    """T = T0 + U(-amp, amp) and C = C0 + U(-amp, amp) at every node.  All of T is drawn
    first, then all of C, row-major (x fastest)."""
    rng = np.random.default_rng(seed)
    T = T0 + rng.uniform(-amp, amp, size=(ny, nx))
    C = C0 + rng.uniform(-amp, amp, size=(ny, nx))
    return T, C


def grf_porosity(nx: int, ny: int, seed, ell: float = 32.0, lo: float = 0.3, hi: float = 0.8):
    """Porosity from a periodic Gaussian random field with covariance exp(-r^2 / (2 ell^2)),
    synthesised by FFT from white noise, standardised, and mapped through the normal CDF
    to a uniform marginal on [lo, hi]."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((ny, nx))
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    # spectral density of a squared-exponential covariance is ~ exp(-k^2 ell^2 / 2);
    # the filter is its square root
    filt = np.exp(-0.25 * k2 * ell * ell)
    z = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    z = (z - z.mean()) / z.std()
    return lo + (hi - lo) * ndtr(z)


def band_porosity(nx: int, ny: int, seed, nbands: int = 8, lo: float = 0.35, hi: float = 0.9):
    """Porosity layered in ``nbands`` horizontal bands of ny/nbands rows (the last band takes
    any remainder); band b has porosity U[lo, hi], drawn in order b = 0, 1, ..."""
    rng = np.random.default_rng(seed)
    vals = rng.uniform(lo, hi, size=nbands)
    rows = np.minimum(np.arange(ny) * nbands // ny, nbands - 1)
    return np.repeat(vals[rows][:, None], nx, axis=1)


def cavity_params(**kw) -> dict:
    """Problem statement of one cavity with the constants of section 4 as defaults."""
    p = dict(nx=64, ny=64, sides=CAVITY_SIDES, Ra=1e4, Pr=1.0, Le=2.0, Da=1e-2, N=1.0,
             J=1.0, sigma=1.0, phi=0.6, Ma=0.1, varpi=0.0, rho0=1.0,
             Th=1.0, Tl=0.0, Ch=1.0, Cl=0.0)
    p.update(kw)
    return p


def small_cavity(seed: int = 0):
    """64x64 uniform porous cavity (phi = 0.6, Da = 1e-2, Ra = 1e4, Pr = 1, Le = 2, N = 1),
    u = 0 and T = C = 0.5 plus noise of amplitude 1e-3; 5000 steps."""
    p = cavity_params(nx=64, ny=64, Ra=1e4, Da=1e-2, Pr=1.0, Le=2.0, N=1.0, phi=0.6)
    T, C = noise_fields(64, 64, seed)
    return dict(params=p, phi=None, T=T, C=C, steps=5000, name="cavity64_phi0.6_Ra1e4")


def grf_cavity(seed: int = 1, n: int = 512):
    """n x n cavity with a Gaussian-random-field porosity on [0.3, 0.8] (correlation length
    32 cells), Ra = 1e6, Da = 1e-3, Pr = 1, Le = 5, N = -0.5 (opposing); 50000 steps."""
    p = cavity_params(nx=n, ny=n, Ra=1e6, Da=1e-3, Pr=1.0, Le=5.0, N=-0.5, phi=0.55)
    phi = grf_porosity(n, n, seed, ell=32.0, lo=0.3, hi=0.8)
    T, C = noise_fields(n, n, seed)
    return dict(params=p, phi=phi, T=T, C=C, steps=50000, name=f"cavity{n}_grf_Ra1e6")


def band_cavity(seed: int = 2, n: int = 2048):
    """n x n cavity, porosity in 8 horizontal bands drawn from U[0.35, 0.9], Ra = 1e7,
    Da = 1e-4, Pr = 0.7, Le = 10, N = 2; 20000 steps."""
    p = cavity_params(nx=n, ny=n, Ra=1e7, Da=1e-4, Pr=0.7, Le=10.0, N=2.0, phi=0.6)
    phi = band_porosity(n, n, seed, nbands=8, lo=0.35, hi=0.9)
    T, C = noise_fields(n, n, seed)
    return dict(params=p, phi=phi, T=T, C=C, steps=20000, name=f"cavity{n}_bands_Ra1e7")


SWEEP_SIDES = tuple(range(64, 513, 32))   # 64, 96, ..., 512


def sweep_cavities(count: int = 256, seed: int = 3):
    """Independent cavities for a batched sweep.  Per cavity, in order: side length from
    {64, 96, ..., 512}, aspect ratio 1 or 2 (ny = A nx), Ra log-uniform [1e3, 1e6], Da
    log-uniform [1e-4, 1e-1], porosity U[0.3, 0.9], Le U[1, 10], N U[-2, 2]; Pr = 1.
    Initial noise uses the seed (seed, index)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        side = int(rng.choice(SWEEP_SIDES))
        A = int(rng.choice((1, 2)))
        Ra = float(10 ** rng.uniform(3, 6))
        Da = float(10 ** rng.uniform(-4, -1))
        phi = float(rng.uniform(0.3, 0.9))
        Le = float(rng.uniform(1, 10))
        N = float(rng.uniform(-2, 2))
        p = cavity_params(nx=side, ny=A * side, Ra=Ra, Da=Da, Pr=1.0, Le=Le, N=N, phi=phi)
        out.append(dict(params=p, noise_seed=(seed, i)))
    return out


def cavity_fields(entry: dict):
    """Initial T, C (noise) of a sweep or request entry."""
    p = entry["params"]
    return noise_fields(p["nx"], p["ny"], list(entry["noise_seed"]))


def request_stream(count: int = 10000, seed: int = 4, rate: float = 1.0,
                   sizes=(128, 256, 512, 1024), probs=(0.4, 0.3, 0.2, 0.1)):
    """Solve requests arriving as a Poisson stream of the given rate (per second).
    Each request: arrival time, square side drawn from ``sizes`` with ``probs``,
    physical parameters drawn as in ``sweep_cavities`` and a storage precision,
    FP32 or FP16 storage, 50/50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        side = int(rng.choice(sizes, p=probs))
        Ra = float(10 ** rng.uniform(3, 6))
        Da = float(10 ** rng.uniform(-4, -1))
        phi = float(rng.uniform(0.3, 0.9))
        Le = float(rng.uniform(1, 10))
        N = float(rng.uniform(-2, 2))
        prec = "fp32" if rng.uniform() < 0.5 else "fp16s"
        p = cavity_params(nx=side, ny=side, Ra=Ra, Da=Da, Pr=1.0, Le=Le, N=N, phi=phi)
        out.append(dict(id=i, arrival=t, params=p, precision=prec, noise_seed=(seed, i)))
    return out


def lattice_updates(nx: int, ny: int, steps: int) -> int:
    return int(nx) * int(ny) * int(steps)


def sample_nodes(nx: int, ny: int, count: int = 2048, seed: int = 12345):
    """``count`` distinct lattice nodes drawn uniformly without replacement (seeded), as
    (x, y) integer arrays: the nodes at which a stored reference keeps its fields."""
    rng = np.random.default_rng(seed)
    k = rng.choice(nx * ny, size=min(count, nx * ny), replace=False)
    k.sort()
    return (k % nx).astype(np.int64), (k // nx).astype(np.int64)


def band_rows(ny: int, nbands: int = 8):
    """Row index ranges [start, stop) of ``nbands`` horizontal bands (the last takes any
    remainder), as used by ``band_porosity``."""
    rows = np.minimum(np.arange(ny) * nbands // ny, nbands - 1)
    return [(int(np.flatnonzero(rows == b)[0]), int(np.flatnonzero(rows == b)[-1]) + 1) for b in range(nbands)]
