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


# ------------------------------------------------------ batched and serving
def batch_grids(count: int = 256, seed: int = 0, nmin: int = 32, nmax: int = 512) -> list:
    """Independent periodic grids of uneven size for the batched form: sides
    log-uniform in [nmin, nmax], 1-4 tanh circles with radii 5-25 % of the
    shorter side (union by max), and half the grids in uniform flow (random
    angle, |u| <= 0.05), half in rotation about the grid centre (largest
    speed, at the corners, <= 0.05); upwind-3, W = 4, M = 0.01, C = 0.5.
    phi0 is drawn by `batch_phi0(grid)`."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(nmin), math.log(nmax)
    out = []
    for k in range(count):
        nx = int(round(math.exp(rng.uniform(lo, hi))))
        ny = int(round(math.exp(rng.uniform(lo, hi))))
        m = min(nx, ny)
        ncirc = int(rng.integers(1, 5))
        cseed = int(rng.integers(0, 2 ** 31 - 1))
        if rng.random() < 0.5:
            ang, sp = rng.uniform(0.0, 2 * math.pi), rng.uniform(0.0, 0.05)
            kind, prm = VEL_UNIFORM, (sp * math.cos(ang), sp * math.sin(ang))
        else:
            umax = rng.uniform(0.0, 0.05)
            omega = umax / math.hypot(nx / 2, ny / 2)
            kind, prm = VEL_ROTATION, (omega, nx / 2, ny / 2)
        out.append(dict(nx=nx, ny=ny, mobility=0.01, width=4.0, cfl=0.5, recon=UPWIND3,
                        vel_kind=kind, vel_param=prm, circles=ncirc, rmin=0.05 * m,
                        rmax=0.25 * m, seed=cseed, steps=2000))
    return out


def batch_phi0(g: dict) -> np.ndarray:
    return random_circles(g["nx"], g["ny"], g["circles"], g["rmin"], g["rmax"],
                          g["width"], g["seed"])


def serve_trace(count: int = 1000, rate: float = 200.0, nmin: int = 64, nmax: int = 4096,
                smin: int = 500, smax: int = 20000, seed: int = 0) -> list:
    """Request stream of interface-tracking solves: Poisson arrivals (mean
    `rate` per second), square grids with sides log-uniform in [nmin, nmax],
    step counts uniform in [smin, smax].  Half the requests are a single vortex
    (U0 = 0.05, modulated by cos(pi t / (steps dt)) so that the flow reverses
    at half time; circle R = 0.15 N at (0.5 N, 0.75 N), not wrapped), half a
    rigid rotation about the centre with corner speed 0.05 (circle R = 0.15 N
    at (0.5 N, 0.65 N), periodic); upwind-3, W = 4, M = 0.01, C = 0.5."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(nmin), math.log(nmax)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(lo, hi))))
        steps = int(rng.integers(smin, smax + 1))
        cfl = 0.5
        if rng.random() < 0.5:
            kind, prm = VEL_SINGLE_VORTEX, (0.05, steps * cfl)
            circle = (0.5 * n, 0.75 * n, 0.15 * n, False)
        else:
            kind, prm = VEL_ROTATION, (0.05 / (math.sqrt(2.0) * n / 2), n / 2, n / 2)
            circle = (0.5 * n, 0.65 * n, 0.15 * n, True)
        out.append(dict(id=k, arrival=t, nx=n, ny=n, steps=steps, mobility=0.01, width=4.0,
                        cfl=cfl, recon=UPWIND3, vel_kind=kind, vel_param=prm, circle=circle))
    return out


def tanh_circle_torch(nx: int, ny: int, cx: float, cy: float, radius: float, width: float,
                      periodic: bool, device) -> "torch.Tensor":
    """tanh_circle drawn directly in device memory (FP64), for requests whose
    phi0 is too large to draw on the host at arrival rate."""
    import torch
    x = torch.arange(nx, dtype=torch.float64, device=device) + 0.5 - cx
    y = torch.arange(ny, dtype=torch.float64, device=device) + 0.5 - cy
    if periodic:
        x = x - nx * torch.round(x / nx)
        y = y - ny * torch.round(y / ny)
    r = torch.sqrt(y[:, None] ** 2 + x[None, :] ** 2)
    return 0.5 + 0.5 * torch.tanh(2.0 * (radius - r) / width)
