"""Seeded synthetic inputs for the k-space-preconditioned PDHG hot path.

This module generates *inputs only*: images, coil sensitivity maps, k-space
trajectories and noise.  It holds none of the reconstruction arithmetic (no
Fourier operator, no preconditioner, no solver), so the FP64 oracle and the
HIP path can both take their inputs from here without sharing any of the
method's code.

Conventions shared by every consumer (they describe the data, not the method):

* An image of shape ``(N_0, ..., N_{d-1})`` is stored C-order, last axis
  fastest.  Array index ``m_a`` sits at the centred position
  ``n_a = m_a - N_a // 2``.
* Coil maps are stored coil-major, shape ``(C, *shape)``, and are normalised
  so that ``sum_c |s_c|^2 = 1`` at every voxel.
* Trajectories are float32 arrays of shape ``(M, d)`` in radians per pixel,
  nominally in ``[-pi, pi)``; column ``a`` pairs with image axis ``a``.
* Random streams: ``numpy.random.default_rng`` over
  ``SeedSequence(seed).spawn(4)``, used for phantom, maps, trajectory and
  noise in that order.

The workloads mirror the paper's data (Experiments / Dataset Details): radial
(brain, liver), variable-density spiral (cardiac) and 3D centre-out UTE
radial, with the sizes of the five benchmark configurations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "streams", "phantom", "coil_maps", "radial_2d", "spiral_2d",
    "fibonacci_sphere", "ute_3d", "noise", "random_coords", "Config",
    "CONFIGS", "config", "slice_config4",
]


def streams(seed: int):
    """Four independent generators: phantom, maps, trajectory, noise."""
    ss = np.random.SeedSequence(int(seed)).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def _centred_grid(shape):
    """Normalised coordinates r_a = n_a / (N_a/2) in [-1, 1) for each axis."""
    axes = [(np.arange(n) - n // 2) / (n / 2.0) for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def _rotation(d: int, rng) -> np.ndarray:
    if d == 2:
        a = rng.uniform(0.0, math.pi)
        return np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    q = q * np.sign(np.diag(r))
    return q


def phantom(shape, rng, n_ellipses: int = 10) -> np.ndarray:
    """Sum of random complex-valued ellipses (2D) or ellipsoids (3D).

    Centre ~ U(-0.5, 0.5)^d, semi-axes ~ U(0.1, 0.5)^d, random rotation,
    amplitude ~ U(0.2, 1), phase ~ U(0, 2 pi); normalised to max |x| = 1.
    Returned as complex128.
    """
    shape = tuple(int(n) for n in shape)
    d = len(shape)
    r = np.stack(_centred_grid(shape), axis=-1)  # (*shape, d)
    x = np.zeros(shape, dtype=np.complex128)
    for _ in range(n_ellipses):
        centre = rng.uniform(-0.5, 0.5, size=d)
        axes = rng.uniform(0.1, 0.5, size=d)
        rot = _rotation(d, rng)
        amp = rng.uniform(0.2, 1.0)
        phase = rng.uniform(0.0, 2 * math.pi)
        local = (r - centre) @ rot  # rotate into the ellipse frame
        inside = np.sum((local / axes) ** 2, axis=-1) <= 1.0
        x[inside] += amp * np.exp(1j * phase)
    m = np.abs(x).max()
    if m > 0:
        x /= m
    return x


def fibonacci_sphere(n: int) -> np.ndarray:
    """n deterministic, nearly uniform unit vectors (golden-angle spiral)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (i + 0.5) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def coil_maps(shape, ncoils: int, rng) -> np.ndarray:
    """Smooth Gaussian-blob coil maps with linear phase, unit sum of squares.

    Coil centres sit on a circle of radius 1.2 (2D, jittered angles) or on
    Fibonacci-sphere points scaled by 1.2 (3D).  Magnitude
    exp(-|r - r_c|^2 / (2 w_c^2)) with w_c ~ U(0.6, 1.0); phase
    phi_c + kappa_c . (r - r_c).  Normalised at every voxel so that
    sum_c |s_c|^2 = 1 exactly.  Returns complex128 of shape (C, *shape).
    """
    shape = tuple(int(n) for n in shape)
    d = len(shape)
    r = np.stack(_centred_grid(shape), axis=-1)
    if d == 2:
        ang = 2 * math.pi * np.arange(ncoils) / ncoils + rng.uniform(-0.1, 0.1, ncoils)
        centres = 1.2 * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    else:
        centres = 1.2 * fibonacci_sphere(ncoils)
    maps = np.empty((ncoils,) + shape, dtype=np.complex128)
    for c in range(ncoils):
        w = rng.uniform(0.6, 1.0)
        phi = rng.uniform(0.0, 2 * math.pi)
        kappa = rng.uniform(-math.pi / 2, math.pi / 2, size=d)
        diff = r - centres[c]
        mag = np.exp(-np.sum(diff * diff, axis=-1) / (2 * w * w))
        maps[c] = mag * np.exp(1j * (phi + diff @ kappa))
    sos = np.sqrt(np.sum(np.abs(maps) ** 2, axis=0))
    maps /= sos
    return maps


def radial_2d(n_spokes: int, n_samples: int) -> np.ndarray:
    """Full-diameter radial spokes, theta_s = pi s / S, r_t = -pi + 2 pi t / T."""
    th = math.pi * np.arange(n_spokes) / n_spokes
    rr = -math.pi + 2 * math.pi * np.arange(n_samples) / n_samples
    k0 = np.outer(np.cos(th), rr).ravel()
    k1 = np.outer(np.sin(th), rr).ravel()
    return np.stack([k0, k1], axis=1).astype(np.float32)


def spiral_2d(n_interleaves: int, n_samples: int, n_turns: float) -> np.ndarray:
    """Archimedean spiral interleaves (density ~ 1/|k|).

    k_j(t) = pi t exp(i (2 pi n_turns t + 2 pi j / J)), t = s / n_samples.
    """
    t = np.arange(n_samples) / n_samples
    out = []
    for j in range(n_interleaves):
        k = math.pi * t * np.exp(1j * (2 * math.pi * n_turns * t + 2 * math.pi * j / n_interleaves))
        out.append(np.stack([k.real, k.imag], axis=1))
    return np.concatenate(out, axis=0).astype(np.float32)


def ute_3d(n_spokes: int, n_samples: int) -> np.ndarray:
    """3D centre-out half spokes along Fibonacci-sphere directions.

    r_s = pi s / n_samples, s = 0..n_samples-1; every spoke starts at k = 0,
    so the density falls like 1/|k|^2.
    """
    dirs = fibonacci_sphere(n_spokes)
    r = math.pi * np.arange(n_samples) / n_samples
    k = dirs[:, None, :] * r[None, :, None]
    return k.reshape(-1, 3).astype(np.float32)


def noise(shape, sigma: float, rng) -> np.ndarray:
    """Complex white Gaussian noise with E|w|^2 = sigma^2."""
    return (sigma / math.sqrt(2.0)) * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_coords(m: int, d: int, rng, specials: bool = True) -> np.ndarray:
    """Uniform random coordinates in [-pi, pi)^d plus awkward special points.

    The special points are the exact centre, axis-aligned points with
    exactly-integer grid positions, the float32 value nearest -pi (which lies
    just below -pi) and values just below +pi.
    """
    k = rng.uniform(-math.pi, math.pi, size=(m, d))
    if specials and m >= 8 * d:
        p32 = float(np.float32(math.pi))
        k[0] = 0.0
        k[1] = -p32
        k[2, :] = 0.0
        k[2, 0] = -p32
        k[3] = np.nextafter(np.float32(math.pi), np.float32(0.0))
        k[4, :] = 0.0
        k[4, -1] = math.pi / 2
        k[5, :] = -math.pi / 4
        k[6] = k[0]
        k[7] = k[1]
    return k.astype(np.float32)


@dataclass
class Config:
    """One benchmark workload: sizes, trajectory recipe and solver settings."""
    name: str
    shape: tuple
    ncoils: int
    alpha: float
    width: int
    reg: str                    # "l2" or "l1wav"
    lam: float
    precond: str                # "sc" or "mc"
    iters: int
    sigma_noise: float = 1e-3
    traj: Optional[dict] = None
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    def coords(self, rng=None) -> np.ndarray:
        t = self.traj
        if t["kind"] == "radial":
            return radial_2d(t["spokes"], t["samples"])
        if t["kind"] == "spiral":
            return spiral_2d(t["interleaves"], t["samples"], t["turns"])
        if t["kind"] == "ute":
            return ute_3d(t["spokes"], t["samples"])
        raise ValueError(t["kind"])

    def inputs(self, seed: int):
        """(x, maps or None, coords, noise) for this configuration."""
        rp, rm, rt, rn = streams(seed)
        x = phantom(self.shape, rp)
        maps = None if self.ncoils == 1 and self.extra.get("unit_maps", False) else coil_maps(self.shape, self.ncoils, rm)
        k = self.coords(rt)
        w = noise((self.ncoils, k.shape[0]), self.sigma_noise, rn)
        return x, maps, k, w


CONFIGS = {
    1: Config("2d-radial-128-1coil", (128, 128), 1, 2.0, 4, "l2", 1e-3, "sc", 20,
              traj={"kind": "radial", "spokes": 64, "samples": 256}, extra={"unit_maps": True}),
    2: Config("2d-spiral-256-8coil", (256, 256), 8, 1.25, 4, "l1wav", 5e-3, "mc", 30,
              traj={"kind": "spiral", "interleaves": 32, "samples": 2048, "turns": 4.0}),
    3: Config("3d-ute-160-8coil", (160, 160, 160), 8, 1.25, 4, "l1wav", 5e-3, "mc", 30,
              traj={"kind": "ute", "spokes": 20000, "samples": 128}),
    5: Config("2d-spiral-256-12coil-unrolled", (256, 256), 12, 1.25, 4, "l2", 1e-3, "mc", 10,
              traj={"kind": "spiral", "interleaves": 24, "samples": 2048, "turns": 16.0 / 3.0},
              extra={"batch": 8}),
}


def config(i: int) -> Config:
    return CONFIGS[i]


def slice_config4(n_slices: int = 64, seed: int = 4, ncoils: int = 12):
    """Per-slice sizes of the batched workload: uneven images and spoke counts.

    N ~ U{128, 192, 256, 320}, S ~ U{32..256} spokes of 2N samples each,
    theta_s = pi s / S, r_t = -pi + 2 pi t / (2N).  Returns a list of
    (shape, coords) pairs; images, maps and noise come from ``streams`` per
    slice (seed * 1000 + slice index).
    """
    rt = streams(seed)[2]
    out = []
    for _ in range(n_slices):
        n = int(rt.choice([128, 192, 256, 320]))
        s = int(rt.integers(32, 257))
        out.append(((n, n), radial_2d(s, 2 * n)))
    return out
