"""Seeded synthetic inputs for the KB-NUFFT path.

This module only draws inputs: trajectories (sampling locations omega, in
radians per voxel), images, coil sensitivity maps and upstream gradients.  It
contains none of the NUFFT arithmetic, so the CPU oracle and the GPU path can
both consume its arrays without sharing any of the method's code.

The shapes follow the paper's workloads: 2D radial spokes through the k-space
centre (the accuracy experiment of Sec. IV-A uses one radial spoke), variable
density spiral interleaves (16 interleaves x 1280 samples, the trajectory
learning experiments of Sec. IV-B), 3D radial "kooshball" spokes and smooth
multi-coil sensitivity maps (the SENSE model of Sec. II-G).  The paper's own
images (fastMRI, Shepp-Logan crop) and ESPIRiT maps are replaced by seeded
Gaussian noise images and Gaussian-bump maps of the same shapes.

All generators return numpy arrays: omega as float32 [M, D] (column d pairs
with image axis d, axis 0 slowest), images as complex64 in row-major order.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def radial_2d(spokes: int, samples: int, jitter: float = 0.0, seed: int = 0) -> np.ndarray:
    """Golden-angle radial trajectory, spoke s at angle s*pi/phi.

    Sample k of a spoke sits at radius pi*(2k - R)/R, so spokes cover
    [-pi, pi) and all pass through the origin.  ``jitter`` adds a uniform
    offset in [-jitter, jitter) radians to every coordinate, after which
    coordinates are wrapped back into [-pi, pi).
    """
    s = np.arange(spokes, dtype=np.float64)[:, None]
    k = np.arange(samples, dtype=np.float64)[None, :]
    theta = s * math.pi / GOLDEN
    rho = math.pi * (2.0 * k - samples) / samples
    om = np.stack([rho * np.cos(theta), rho * np.sin(theta)], axis=-1).reshape(-1, 2)
    if jitter:
        om = om + rng(seed).uniform(-jitter, jitter, size=om.shape)
        om = np.mod(om + math.pi, 2.0 * math.pi) - math.pi
    return om.astype(np.float32)


def spiral_2d(interleaves: int, samples: int, turns: float = 10.0, power: float = 1.5) -> np.ndarray:
    """Variable-density Archimedean-like spiral.

    tau = s/S, radius pi*tau**power, angle 2*pi*turns*tau + 2*pi*q/Q.
    """
    q = np.arange(interleaves, dtype=np.float64)[:, None]
    s = np.arange(samples, dtype=np.float64)[None, :]
    tau = s / samples
    rho = math.pi * tau ** power
    theta = 2.0 * math.pi * turns * tau + 2.0 * math.pi * q / interleaves
    om = np.stack([rho * np.cos(theta), rho * np.sin(theta)], axis=-1).reshape(-1, 2)
    return om.astype(np.float32)


def kooshball_3d(spokes: int, samples: int) -> np.ndarray:
    """3D radial spokes with directions on a golden spiral over a hemisphere."""
    s = np.arange(spokes, dtype=np.float64)
    z = (s + 0.5) / spokes
    phi = 2.0 * math.pi * s * (1.0 - 1.0 / GOLDEN)
    rxy = np.sqrt(1.0 - z * z)
    dirs = np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=-1)
    k = np.arange(samples, dtype=np.float64)
    rho = math.pi * (2.0 * k - samples) / samples
    om = (dirs[:, None, :] * rho[None, :, None]).reshape(-1, 3)
    return om.astype(np.float32)


def uniform_random(M: int, D: int, seed: int, lo: float = -math.pi, hi: float = math.pi) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=(M, D)).astype(np.float32)


def complex_normal(shape, seed: int) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0, 1)."""
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im).astype(np.complex64)


def sense_maps(C: int, N) -> np.ndarray:
    """Smooth Gaussian-bump coil maps, one bump per coil around the FOV.

    Coil c is centred at 0.5*(N/2)*(cos 2pi c/C, sin 2pi c/C) (in 3D the last
    axis centre alternates between +N/4 and -N/4), has width 0.35*N and a
    constant phase 2*pi*c/C.
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) - n // 2 for n in N], indexing="ij")
    out = np.empty((C,) + N, dtype=np.complex64)
    width = 0.35 * max(N)
    for c in range(C):
        ang = 2.0 * math.pi * c / C
        centre = [0.0] * D
        centre[0] = 0.5 * (N[0] / 2.0) * math.cos(ang)
        if D >= 2:
            centre[1] = 0.5 * (N[1] / 2.0) * math.sin(ang)
        if D >= 3:
            centre[2] = (N[2] / 4.0) * (1 if c % 2 == 0 else -1)
        d2 = sum((g - p) ** 2 for g, p in zip(grids, centre))
        out[c] = (np.exp(-d2 / (2.0 * width * width)) * np.exp(1j * ang)).astype(np.complex64)
    return out


def field_map(N, peak_hz: float = 60.0, seed: int = 0) -> np.ndarray:
    """Smooth off-resonance map in rad/s (float32 [*N]): a positive and a
    negative Gaussian bump (width 0.2 max N) at seeded positions plus a
    linear ramp along axis 0, scaled so that the largest |w| is 2 pi peak_hz
    (a shimmed head at 3 T has tens of Hz)."""
    N = tuple(int(n) for n in N)
    g = rng(seed)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) - n // 2 for n in N], indexing="ij")
    width = 0.2 * max(N)
    out = 0.3 * grids[0] / max(1, N[0] // 2)
    for sign in (1.0, -1.0):
        centre = [g.uniform(-0.3, 0.3) * n for n in N]
        d2 = sum((x - p) ** 2 for x, p in zip(grids, centre))
        out = out + sign * np.exp(-d2 / (2.0 * width * width))
    out = out / max(1e-12, np.abs(out).max())
    return (2.0 * math.pi * peak_hz * out).astype(np.float32)


def readout_times(interleaves: int, samples: int, dwell: float = 4e-6, t0: float = 0.0) -> np.ndarray:
    """Readout time of every sample (float32 [interleaves * samples], s):
    each interleave is read out from t0 with a constant dwell time, matching
    the sample order of ``spiral_2d`` and ``radial_2d``."""
    s = t0 + dwell * np.arange(samples, dtype=np.float64)
    return np.tile(s, interleaves).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-shaped configurations)
# ---------------------------------------------------------------------------

def small_radial_case(seed: int = 1001):
    """64x64 image, 32 golden-angle spokes x 128 samples (M = 4096)."""
    N = (64, 64)
    om = radial_2d(32, 128)
    x = complex_normal(N, seed)
    return N, om, x


def throughput_case(batch: int, seed: int = 2001):
    """256x256 images, 64 spokes x 512 samples (M = 32768) with +-pi/N jitter."""
    N = (256, 256)
    om = radial_2d(64, 512, jitter=math.pi / 256, seed=seed)
    x = complex_normal((batch,) + N, seed + 1)
    return N, om, x


def spiral_sense_case(batch: int = 8, coils: int = 8, seed: int = 3001):
    """320x320 images, 8 coils, 16 spiral interleaves x 1280 samples (M = 20480)."""
    N = (320, 320)
    om = spiral_2d(16, 1280)
    x = complex_normal((batch,) + N, seed)
    smaps = sense_maps(coils, N)
    return N, om, x, smaps


def multi_instance_case(n2d: int = 32, seed: int = 4001, n_range=(128, 384),
                        m_range=(8000, 80000), coil_range=(4, 8),
                        shape3d=(128, 128, 128), spokes3d: int = 4096, samples3d: int = 256):
    """Uneven SENSE problems sharing one GPU.

    n2d 2D instances with N_d drawn independently per axis from n_range,
    M from m_range and the coil count from coil_range (all inclusive);
    even-numbered instances use golden-angle radial spokes of 2 max(N)
    samples, odd-numbered ones 16 spiral interleaves, truncated to M
    samples.  Then one 3D kooshball instance of shape3d with one coil
    (spokes3d x samples3d samples), unless shape3d is None.
    Returns a list of dicts with keys N, omega, coils, kind.
    """
    g = rng(seed)
    out = []
    for i in range(n2d):
        N = tuple(int(v) for v in g.integers(n_range[0], n_range[1] + 1, size=2))
        M = int(g.integers(m_range[0], m_range[1] + 1))
        C = int(g.integers(coil_range[0], coil_range[1] + 1))
        if i % 2 == 0:
            R = 2 * max(N)
            om = radial_2d(-(-M // R), R)[:M]
            kind = "radial"
        else:
            om = spiral_2d(16, -(-M // 16))[:M]
            kind = "spiral"
        out.append({"N": N, "omega": np.ascontiguousarray(om), "coils": C, "kind": kind})
    if shape3d is not None:
        out.append({"N": tuple(shape3d), "omega": kooshball_3d(spokes3d, samples3d), "coils": 1,
                    "kind": "kooshball"})
    return out


def instance_data(inst: dict, seed: int):
    """Image [1, *N], coil maps [C, *N] (None for one coil) and a k-space
    array [1, C, M] (upstream gradient or data) for one instance."""
    N, C, M = inst["N"], inst["coils"], inst["omega"].shape[0]
    x = complex_normal((1,) + tuple(N), seed)
    smaps = sense_maps(C, N) if C > 1 else None
    k = complex_normal((1, C, M), seed + 1)
    return x, smaps, k
