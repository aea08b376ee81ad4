"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the lattice Boltzmann method itself: it
only turns a seed into the initial density field the method starts from.
Both the CPU oracle and the HIP library receive the same array, so neither
side re-implements the other's random numbers.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), evaluated counter-style: the i-th draw is
the SplitMix64 output for state ``seed + (i + 1) * golden_gamma``.  The top
53 bits give a double in [0, 1).
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given 0-based counters (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counters.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from counters start..start+n-1 (top 53 bits)."""
    c = np.arange(start, start + n, dtype=np.uint64)
    z = splitmix64(seed, c)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def noisy_density(nx: int, ny: int, nz: int, rho_mean: float, noise_amp: float,
                  seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """rho0[k, j, i] = rho_mean * (1 + a * (2u - 1)), u i.i.d. U[0,1) per node.

    The node counter is i + nx * (j + ny * k), so the field is the same for
    any chunking.  Returned as a C-contiguous float64 array of shape
    (nz, ny, nx).
    """
    n = nx * ny * nz
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = uniform01(seed, e - s, start=s)
        out[s:e] = rho_mean * (1.0 + noise_amp * (2.0 * u - 1.0))
    return out.reshape(nz, ny, nx)


def random_unit_field(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """A seeded direction in field space (unit 2-norm), for directional
    derivative checks."""
    u = uniform01(seed, nx * ny * nz) * 2.0 - 1.0
    u /= np.linalg.norm(u)
    return u.reshape(nz, ny, nx)


def bubbly_density(n: int, rho_g: float, rho_l: float, n_bubbles: int, r_min: float,
                   r_max: float, seed: int, width: float = 2.0) -> np.ndarray:
    """A periodic n^3 liquid of density rho_l holding n_bubbles spherical
    bubbles of density rho_g: centres uniform in the box, radii uniform in
    [r_min, r_max], each a tanh profile of the given width (minimum-image
    distance); where bubbles overlap the lower density wins.  Shape (n, n, n),
    float64."""
    u = uniform01(seed, 4 * n_bubbles).reshape(n_bubbles, 4)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    out = np.full((n, n, n), rho_l, dtype=np.float64)
    for cx, cy, cz, ur in u:
        c = np.array([cx, cy, cz]) * n
        R = r_min + (r_max - r_min) * ur
        d2 = np.zeros_like(out)
        for a, ca in ((x, c[0]), (y, c[1]), (z, c[2])):
            da = np.abs(a + 0.5 - ca)
            da = np.minimum(da, n - da)
            d2 += da * da
        prof = rho_g + (rho_l - rho_g) * 0.5 * (1.0 + np.tanh((np.sqrt(d2) - R) / width))
        out = np.minimum(out, prof)
    return out


def noisy_density_at(nx: int, ny: int, nz: int, rho_mean: float, noise_amp: float, seed: int,
                     k: np.ndarray, j: np.ndarray, i: np.ndarray) -> np.ndarray:
    """noisy_density(nx, ny, nz, ...)[k, j, i] for broadcastable index arrays,
    without generating the whole field (same counters, same values)."""
    k, j, i = np.broadcast_arrays(np.asarray(k, dtype=np.uint64), np.asarray(j, dtype=np.uint64),
                                  np.asarray(i, dtype=np.uint64))
    c = i + np.uint64(nx) * (j + np.uint64(ny) * k)
    u = (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return rho_mean * (1.0 + noise_amp * (2.0 * u - 1.0))
