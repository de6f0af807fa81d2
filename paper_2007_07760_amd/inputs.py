"""Seeded synthetic inputs: initial order-parameter fields and velocity choices.

This module holds none of the scheme's arithmetic: it only draws the initial
phi0 fields and the prescribed-velocity parameters of the paper's workloads
(Sec. III: tanh interfaces of Eq. (3), a sharp slotted disk, periodic grids of
unit cells) so that the HIP path and the oracle can be fed the same arrays.
Cell (x, y) has its centre at (x + 1/2, y + 1/2).
"""
from __future__ import annotations

import math

import numpy as np

# velocity kinds of the C ABI (same numbering as include/dugks.h)
VEL_UNIFORM, VEL_ROTATION, VEL_SINGLE_VORTEX, VEL_DEFORMATION, VEL_ARRAYS = range(5)
CENTRAL2, UPWIND3, CENTRAL4 = 0, 1, 2


def _centres(nx: int, ny: int):
    x = np.arange(nx, dtype=np.float64) + 0.5
    y = np.arange(ny, dtype=np.float64) + 0.5
    return np.meshgrid(x, y)  # arrays [y][x]


def _periodic_delta(d: np.ndarray, n: int) -> np.ndarray:
    return d - n * np.round(d / n)


def tanh_circle(nx: int, ny: int, cx: float, cy: float, radius: float,
                width: float, periodic: bool = True) -> np.ndarray:
    """phi = 1/2 + 1/2 tanh(2 (R - r) / W): phase A (phi = 1) inside (Eq. 3)."""
    X, Y = _centres(nx, ny)
    dx, dy = X - cx, Y - cy
    if periodic:
        dx, dy = _periodic_delta(dx, nx), _periodic_delta(dy, ny)
    r = np.sqrt(dx * dx + dy * dy)
    return 0.5 + 0.5 * np.tanh(2.0 * (radius - r) / width)


def tanh_circles(nx: int, ny: int, centres, radii, width: float) -> np.ndarray:
    """Union (pointwise max) of several periodic tanh circles."""
    out = np.zeros((ny, nx))
    for (cx, cy), r in zip(centres, radii):
        out = np.maximum(out, tanh_circle(nx, ny, cx, cy, r, width))
    return out


def random_circles(nx: int, ny: int, count: int, rmin: float, rmax: float,
                   width: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = [(rng.uniform(0, nx), rng.uniform(0, ny)) for _ in range(count)]
    radii = [rng.uniform(rmin, rmax) for _ in range(count)]
    return tanh_circles(nx, ny, centres, radii, width)


def slotted_disk(nx: int, ny: int, cx: float, cy: float, radius: float,
                 slot_w: float, slot_depth: float) -> np.ndarray:
    """Sharp 0/1 slotted disk sampled at cell centres; the slot is cut upward
    from the bottom of the disk, slot_w wide and slot_depth deep."""
    X, Y = _centres(nx, ny)
    inside = (X - cx) ** 2 + (Y - cy) ** 2 <= radius ** 2
    bottom = cy - radius
    slot = (np.abs(X - cx) <= 0.5 * slot_w) & (Y <= bottom + slot_depth)
    return (inside & ~slot).astype(np.float64)


def planar_slab(nx: int, ny: int, half_width: float, width: float) -> np.ndarray:
    """Slab of phase A centred at x = nx/2, flat tanh interfaces normal to x."""
    X, _ = _centres(nx, ny)
    return 0.5 + 0.5 * np.tanh(2.0 * (half_width - np.abs(X - 0.5 * nx)) / width)


def cosine_mode(nx: int, ny: int, amp: float, kx: int, ky: int) -> np.ndarray:
    """phi = 1/2 + amp cos(2 pi (kx x / nx + ky y / ny))."""
    X, Y = _centres(nx, ny)
    return 0.5 + amp * np.cos(2.0 * math.pi * (kx * X / nx + ky * Y / ny))


def random_smooth(nx: int, ny: int, seed: int, modes: int = 4) -> np.ndarray:
    """A smooth periodic random field in (0, 1) made of a few Fourier modes."""
    rng = np.random.default_rng(seed)
    X, Y = _centres(nx, ny)
    out = np.full((ny, nx), 0.5)
    for _ in range(modes):
        kx, ky = rng.integers(-3, 4, size=2)
        a = rng.uniform(0.02, 0.1)
        ph = rng.uniform(0, 2 * math.pi)
        out += a * np.cos(2 * math.pi * (kx * X / nx + ky * Y / ny) + ph)
    return out


# --------------------------------------------------------------- workloads
def workload(name: str, seed: int = 0) -> dict:
    """Named synthetic workloads: the parameters of each solve and its phi0.

    c1      64^2 FP64 central-2 translating circle (one period = 3200 steps)
    c2      256^2 upwind-3 slotted disk in rigid rotation (8000 steps/turn)
    c3_512  512^2 single vortex, stretch to T and back at 2T
    h1      4096^2 upwind-3, 64 random tanh circles in rigid rotation
    """
    if name == "c1":
        n = 64
        return dict(nx=n, ny=n, mobility=0.01, width=4.0, cfl=0.5, recon=CENTRAL2,
                    vel_kind=VEL_UNIFORM, vel_param=(0.04, 0.04),
                    phi0=tanh_circle(n, n, 32.0, 32.0, 16.0, 4.0), steps=3200)
    if name == "c2":
        n = 256
        omega = 2 * math.pi / (8000 * 0.5)
        return dict(nx=n, ny=n, mobility=0.005, width=4.0, cfl=0.5, recon=UPWIND3,
                    vel_kind=VEL_ROTATION, vel_param=(omega, 128.0, 128.0),
                    phi0=slotted_disk(n, n, 128.0, 160.0, 50.0, 12.0, 60.0),
                    steps=8000)
    if name.startswith("c3"):
        n = int(name.split("_")[1]) if "_" in name else 512
        u0, cfl = 0.08, 0.5
        T = n / (2 * u0)
        steps = int(round(2 * T / cfl))
        return dict(nx=n, ny=n, mobility=0.02, width=4.0, cfl=cfl, recon=UPWIND3,
                    vel_kind=VEL_SINGLE_VORTEX, vel_param=(u0, 2 * T),
                    phi0=tanh_circle(n, n, 0.5 * n, 0.75 * n, 0.15 * n, 4.0,
                                     periodic=False),
                    steps=steps)
    if name == "h1":
        n = 4096
        umax = 0.05
        omega = umax / (math.sqrt(2.0) * n / 2)   # corner speed = umax
        return dict(nx=n, ny=n, mobility=0.01, width=4.0, cfl=0.5, recon=UPWIND3,
                    vel_kind=VEL_ROTATION, vel_param=(omega, n / 2, n / 2),
                    phi0=random_circles(n, n, 64, 20.0, 200.0, 4.0, seed),
                    steps=200)
    raise KeyError(name)
