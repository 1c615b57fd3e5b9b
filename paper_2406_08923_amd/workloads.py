"""Coefficient tensors of the benchmark workloads, built from the library's own
finite-difference weights (stencil_fd_weights).

* smoother3: the 1-D radius-1 stencil [1/4, 1/2, 1/4]; Eq. 5 with the second
  difference [1, -2, 1] and alpha*dt/ds^2 = 1/4.
* laplacian_star(ndim, r): the (2r)-th order central Laplacian in grid units,
  summed over the axes (Eq. 6-7): 6r+1 nonzero taps in 3-D.
* diffusion_star(ndim, r, s): one forward-Euler diffusion step as a single
  cross-correlation (Eq. 5, Eq. 7): identity + s * laplacian_star.
"""
import math

import numpy as np

from . import fd_weights


def smoother3():
    return np.array([0.25, 0.5, 0.25])


def laplacian_star(ndim, r):
    c = fd_weights(2, r)
    g = np.zeros((2 * r + 1,) * ndim)
    for a in range(ndim):
        idx = [r] * ndim
        for m in range(-r, r + 1):
            idx[a] = r + m
            g[tuple(idx)] += c[m + r]
    return g


def diffusion_star(ndim, r, s):
    g = s * laplacian_star(ndim, r)
    g[(r,) * ndim] += 1.0
    return g


def diffusion_number(n, alpha=1.0, dt_factor=1e-3):
    """s = alpha dt / ds^2 with ds = 2 pi / n and dt = dt_factor * ds (the
    diffusion setup of Table B2)."""
    ds = 2.0 * math.pi / n
    return alpha * dt_factor * ds / ds ** 2


def aligned_layout(nx, r, elem_bytes, line=128):
    """(row_pitch, x_offset) that start the interior of every row on a
    ``line``-byte boundary: x_offset is the smallest multiple of the line
    (in elements) that is >= r, the pitch the smallest multiple >= x_offset +
    nx + r. Allocations from the HIP allocator are at least 256-byte
    aligned, so every interior row then starts a cache line."""
    per = max(1, line // elem_bytes)
    ox = -(-r // per) * per
    pitch = -(-(ox + nx + r) // per) * per
    return pitch, ox
