"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws densities; it holds none of the homogenization
arithmetic.  Every generator is a pure function of its arguments, so a test
can hand exactly the same field to the GPU path and to the FP64 oracle.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) evaluated at a counter built
from ``(seed, stream, index)``:

    key = (seed mod 2^24) << 40 | (stream mod 16) << 36 | index,  index < 2^36
    uniform = (splitmix64(key) >> 11) * 2^-53              in [0, 1)

Densities are laid out x-fastest, ``idx = x + nx*(y + ny*z)``, and returned as
numpy arrays of shape ``(nz, ny, nx)`` (C order, so ``.ravel()`` gives idx).
"""
from __future__ import annotations

import math
import os

import numpy as np

try:  # multi-threaded pocketfft; same transform as numpy.fft
    import scipy.fft as _fft
    _FFT_KW = {"workers": min(16, os.cpu_count() or 1)}
except ImportError:  # pragma: no cover
    _fft = np.fft
    _FFT_KW = {}

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to uint64 counters."""
    z = np.asarray(x, dtype=np.uint64) + _GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """``n`` doubles in [0, 1) for counters ``index = 0..n-1`` of (seed, stream)."""
    if n >= (1 << 36):
        raise ValueError("index space of one stream is 2^36")
    key = (np.uint64((seed % (1 << 24)) << 40) | np.uint64((stream % 16) << 36))
    idx = np.arange(n, dtype=np.uint64) | key
    with np.errstate(over="ignore"):
        bits = splitmix64(idx)
    return (bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def standard_normal(seed: int, stream: int, n: int) -> np.ndarray:
    """Box-Muller normals from two uniform streams (``stream`` and ``stream+1``)."""
    u1 = uniform01(seed, stream, n)
    u2 = uniform01(seed, stream + 1, n)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


def uniform_density(shape, seed: int, mean: float = 0.3) -> np.ndarray:
    """I.i.d. uniform[0,1) densities rescaled multiplicatively to the given mean.

    ``shape`` is (nx, ny, nz).  With mean 0.3 the maximum stays near 0.6, so no
    clipping is needed.
    """
    nx, ny, nz = shape
    n = nx * ny * nz
    rho = uniform01(seed, 0, n)
    rho *= mean / rho.mean()
    return rho.reshape(nz, ny, nx)


def _periodic_gauss_1d(length: int, sigma: float) -> np.ndarray:
    """Normalized Gaussian taps truncated at ceil(4 sigma), folded onto a period."""
    r = int(math.ceil(4.0 * sigma))
    k = np.arange(-r, r + 1)
    w = np.exp(-(k.astype(np.float64) ** 2) / (2.0 * sigma * sigma))
    w /= w.sum()
    ker = np.zeros(length)
    np.add.at(ker, k % length, w)
    return ker


def smoothed_noise(shape, seed: int, sigma: float = 3.0) -> np.ndarray:
    """Periodic separable Gaussian smoothing of i.i.d. N(0,1) voxel noise."""
    nx, ny, nz = shape
    v = standard_normal(seed, 2, nx * ny * nz).reshape(nz, ny, nx)
    for axis, length in ((2, nx), (1, ny), (0, nz)):
        ker = np.fft.rfft(_periodic_gauss_1d(length, sigma))
        shp = [1, 1, 1]
        shp[axis] = ker.shape[0]
        spec = _fft.rfft(v, axis=axis, **_FFT_KW)
        spec *= ker.reshape(shp)
        v = _fft.irfft(spec, n=length, axis=axis, **_FFT_KW)
        del spec
    return v


def threshold_top(values: np.ndarray, volfrac: float, floor: float = 1e-3) -> np.ndarray:
    """Exactly round(volfrac*n) voxels with the largest values become 1, the rest ``floor``.

    Ties at the threshold are broken in favour of the lower linear index.
    """
    flat = values.ravel()
    n = flat.size
    k = int(round(volfrac * n))
    out = np.full(n, floor, dtype=np.float64)
    if k <= 0:
        return out.reshape(values.shape)
    if k >= n:
        out[:] = 1.0
        return out.reshape(values.shape)
    t = np.partition(flat, n - k)[n - k]
    above = flat > t
    out[above] = 1.0
    need = k - int(above.sum())
    if need > 0:
        ties = np.flatnonzero(flat == t)[:need]
        out[ties] = 1.0
    return out.reshape(values.shape)


def smoothed_noise_density(shape, seed: int, volfrac: float, sigma: float = 3.0,
                           floor: float = 1e-3) -> np.ndarray:
    """Gaussian-smoothed noise thresholded to a volume fraction (values 1 or floor)."""
    return threshold_top(smoothed_noise(shape, seed, sigma), volfrac, floor)


def box_downsample(rho: np.ndarray, factor: int) -> np.ndarray:
    """Mean over factor^3 blocks of a (nz, ny, nx) field; preserves the mean."""
    nz, ny, nx = rho.shape
    if nx % factor or ny % factor or nz % factor:
        raise ValueError("shape must be divisible by the factor")
    r = rho.reshape(nz // factor, factor, ny // factor, factor, nx // factor, factor)
    return r.mean(axis=(1, 3, 5))


def z_laminate(shape, profile) -> np.ndarray:
    """Density that varies only along z: ``profile[z]`` repeated over each xy plane."""
    nx, ny, nz = shape
    prof = np.asarray(profile, dtype=np.float64)
    if prof.shape != (nz,):
        raise ValueError("profile length must equal nz")
    return np.broadcast_to(prof[:, None, None], (nz, ny, nx)).copy()


def random_signed_field(shape, seed: int, stream: int = 5, ncases: int = 6) -> np.ndarray:
    """Uniform[-1,1) nodal vectors laid out (case, comp, idx): operands for operator tests."""
    nx, ny, nz = shape
    n = nx * ny * nz
    return (2.0 * uniform01(seed, stream, ncases * 3 * n) - 1.0).reshape(ncases, 3, n)


def trig_init_draws(nfreq: int, seed: int):
    """Random draws of the trigonometric initialization: a quaternion with four
    entries in [-1, 1) and one weight in [-1, 1) per basis function of Q_n
    (6 nfreq + 3 nfreq (6 nfreq + 1) functions)."""
    t = 6 * nfreq
    nb = t + t * (t + 1) // 2
    q = 2.0 * uniform01(seed, 13, 4) - 1.0
    w = 2.0 * uniform01(seed, 14, nb) - 1.0
    return q, w
