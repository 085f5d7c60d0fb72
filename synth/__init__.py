"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This module only draws numbers: it holds none of the solver's arithmetic
(no matrix, no CG, no stencil, no convolution of the method). Every array
it returns is a plain numpy array on the host; callers move it where they
need it.

Recipes (the paper uses no dataset; these stand in for its workloads):

* ``uniform_rhs``: i.i.d. uniform[-1, 1] values in x-fastest order from
  ``numpy.random.default_rng(seed)`` (PCG64).
* ``smoothed_rhs``: i.i.d. standard normals from the same generator,
  smoothed by a separable Gaussian of width ``sigma`` cells (truncated at
  four sigma, mirror-reflected at the walls), then shifted to zero mean and
  scaled to unit RMS.  This is the "Gaussian-smoothed random right-hand
  side" workload.
* ``net_init``: He-normal initial weights for the warm-start network, one
  block per layer in tap-major order ``[tap][c_in][c_out]``.
* ``bf16_values``: random values that are exactly representable in
  bfloat16, for kernel-level parity checks.
* ``random_flow``: face velocities on the staggered grid, i.i.d.
  uniform[-amp, amp] from ``default_rng(seed)`` in the order u, v, w, with
  the wall-normal faces set to zero (a flow that exercises every departure
  direction of the advection).

Arrays are indexed ``idx = i + nx * (j + ny * k)`` (x fastest).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_rhs",
    "smoothed_rhs",
    "smoothed_rhs_torch",
    "gaussian_kernel_1d",
    "net_init",
    "net_layer_shapes",
    "bf16_values",
    "bf16_round_np",
    "random_flow",
]


def uniform_rhs(n: int | tuple, seed: int) -> np.ndarray:
    """uniform[-1, 1] values, float64, flat x-fastest array of n^3 (or nx*ny*nz)."""
    if isinstance(n, int):
        count = n * n * n
    else:
        count = int(np.prod(n))
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=count).astype(np.float64)


def gaussian_kernel_1d(sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Normalised 1-D Gaussian taps of radius ceil(truncate*sigma)."""
    radius = int(truncate * sigma + 0.5)
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-0.5 * (t / sigma) ** 2)
    return g / g.sum()


def _smooth_axis(a: np.ndarray, axis: int, taps: np.ndarray) -> np.ndarray:
    from scipy.ndimage import correlate1d
    # mode 'reflect' repeats the edge sample: the mirror about the wall face.
    return correlate1d(a, taps, axis=axis, mode="reflect")


def smoothed_rhs(n: int, seed: int, sigma: float = 3.0) -> np.ndarray:
    """Zero-mean, unit-RMS Gaussian-smoothed white noise on an n^3 grid (float64, flat)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))  # axes (k, j, i): x fastest when flattened
    taps = gaussian_kernel_1d(sigma)
    a = white
    for axis in (2, 1, 0):
        a = _smooth_axis(a, axis, taps)
    a = a - a.mean()
    a = a / np.sqrt(np.mean(a * a))
    return np.ascontiguousarray(a.reshape(-1))


def smoothed_rhs_torch(n: int, seed: int, sigma: float = 3.0, device="cuda"):
    """The smoothed_rhs recipe drawn with torch's generator on `device` (float64).

    Same distribution as smoothed_rhs (different numbers for the same seed):
    for bulk training data, where host generation would dominate.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    a = torch.randn((n, n, n), generator=g, device=device, dtype=torch.float64)
    taps = gaussian_kernel_1d(sigma)
    r = (len(taps) - 1) // 2
    for axis in (2, 1, 0):
        x = a.movedim(axis, 0)
        # mirror about the wall face (edge sample repeated), as scipy 'reflect'
        idx = np.arange(-r, n + r)
        idx = np.where(idx < 0, -idx - 1, idx)
        idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
        while (idx < 0).any() or (idx >= n).any():  # grids smaller than the radius
            idx = np.where(idx < 0, -idx - 1, idx)
            idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
        xp = x[torch.from_numpy(idx).to(x.device)]
        out = torch.zeros_like(x)
        for m, w in enumerate(taps):
            out += float(w) * xp[m:m + n]
        a = out.movedim(0, axis)
    a = a - a.mean()
    a = a / torch.sqrt(torch.mean(a * a))
    return a.reshape(-1).contiguous()


def net_layer_shapes(channels: int = 16, layers: int = 4):
    """(c_in, c_out) per layer of the warm-start network: 1 -> C -> ... -> C -> 1."""
    shapes = []
    for l in range(layers):
        cin = 1 if l == 0 else channels
        cout = 1 if l == layers - 1 else channels
        shapes.append((cin, cout))
    return shapes


def net_init(seed: int, channels: int = 16, layers: int = 4) -> np.ndarray:
    """He-normal weights, float32, concatenated per layer as [27][c_in][c_out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in net_layer_shapes(channels, layers):
        fan_in = 27 * cin
        w = rng.standard_normal((27, cin, cout)) * np.sqrt(2.0 / fan_in)
        parts.append(w.astype(np.float32).reshape(-1))
    return np.concatenate(parts)


def bf16_round_np(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_values(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """float32 array of bfloat16-representable normals (times ``scale``)."""
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal(shape) * scale).astype(np.float32)
    return bf16_round_np(a)


def random_flow(dims, seed: int, amp: float = 1.0):
    """(u, v, w) flat face arrays (x fastest over each component's own face
    grid: (nx+1) x ny x nz, nx x (ny+1) x nz, nx x ny x (nz+1)), uniform in
    [-amp, amp], zero on the wall-normal faces."""
    nx, ny, nz = (dims, dims, dims) if isinstance(dims, int) else dims
    rng = np.random.default_rng(seed)
    u = rng.uniform(-amp, amp, (nz, ny, nx + 1))
    v = rng.uniform(-amp, amp, (nz, ny + 1, nx))
    w = rng.uniform(-amp, amp, (nz + 1, ny, nx))
    u[:, :, 0] = u[:, :, nx] = 0.0
    v[:, 0, :] = v[:, ny, :] = 0.0
    w[0] = w[nz] = 0.0
    return u.reshape(-1), v.reshape(-1), w.reshape(-1)
