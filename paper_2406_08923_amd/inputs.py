"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and samples analytic fields; it holds
none of the stencil arithmetic. The paper benchmarks on randomised arrays and,
for verification, on analytic fields (Sec. 5.1, Table B2); nothing here stands
in for a dataset.

All fields are returned as interior arrays in NumPy order [z, y, x] (x fastest)
without padding.
"""
import math

import numpy as np


def uniform_field(n, seed, lo=-1.0, hi=1.0):
    """Interior field of shape n = (nx[, ny[, nz]]) uniform in [lo, hi)."""
    shape = tuple(int(v) for v in reversed(n))
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def grid_coords(n):
    """Coordinates x_i = 2 pi i / n_i on [0, 2 pi)^d, broadcastable, NumPy order."""
    nd = len(n)
    out = []
    for a in range(nd):
        c = 2.0 * math.pi * np.arange(n[a]) / n[a]
        shape = [1] * nd
        shape[nd - 1 - a] = n[a]
        out.append(c.reshape(shape))
    return out  # [x, y, z]


def draw_modes(rng, count, ndim, kmax, amp):
    """``count`` Fourier modes: integer wavevector with components uniform in
    [-kmax, kmax] (k = 0 redrawn), amplitude amp * U[-1, 1), phase U[0, 2 pi).
    Draw order per mode: k components, amplitude, phase."""
    modes = []
    for _ in range(count):
        while True:
            k = [int(rng.integers(-kmax, kmax + 1)) for _ in range(ndim)]
            if any(k):
                break
        a = amp * float(rng.uniform(-1.0, 1.0))
        ph = float(rng.uniform(0.0, 2.0 * math.pi))
        modes.append((tuple(k), a, ph))
    return modes


def eval_modes(n, modes):
    """sum_m a_m cos(k_m . x + phi_m) on the grid of interior shape n."""
    X = grid_coords(n)
    f = np.zeros(tuple(int(v) for v in reversed(n)))
    for k, a, ph in modes:
        arg = ph
        for ax in range(len(n)):
            arg = arg + k[ax] * X[ax]
        f += a * np.cos(arg)
    return f


def eval_modes_device(n, modes, device="cuda"):
    """eval_modes evaluated with torch on ``device`` (FP64), returned as a
    NumPy array: the same sum of cosines, for grids too large to sample
    quickly on the host (the serving trace's 384^3 jobs)."""
    import torch
    nd = len(n)
    X = []
    for a in range(nd):
        c = 2.0 * math.pi * torch.arange(n[a], dtype=torch.float64, device=device) / n[a]
        shape = [1] * nd
        shape[nd - 1 - a] = n[a]
        X.append(c.reshape(shape))
    f = torch.zeros(tuple(int(v) for v in reversed(n)), dtype=torch.float64, device=device)
    for k, amp, ph in modes:
        arg = torch.full((1,) * nd, ph, dtype=torch.float64, device=device)
        for ax in range(nd):
            arg = arg + k[ax] * X[ax]
        f += amp * torch.cos(arg)
    return f.cpu().numpy()


def fourier_fields(n, seed, nf=8, modes=8, kmax=8, amp=0.01):
    """nf fields, each a sum of ``modes`` random Fourier modes (|k|_inf <= kmax).
    Draw order: field-major, then mode. Returns (list of interior arrays, the
    mode table per field)."""
    rng = np.random.default_rng(seed)
    table = [draw_modes(rng, modes, len(n), kmax, amp) for _ in range(nf)]
    return [eval_modes(n, t) for t in table], table


def to_bf16_values(a):
    """Round a float32/float64 array to the nearest bfloat16 value
    (round-to-nearest-even) and return it widened to float64, so that both the
    oracle and a bf16-storage path see exactly the same input values."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# serving trace
# ---------------------------------------------------------------------------

SERVE_EDGES = (64, 96, 128, 192, 256, 384)


def serving_trace(seed, count, rate=200.0, edges=SERVE_EDGES, steps=(10, 500),
                  p3d=0.5, p_f32=0.5, nu=1e-3, modes=4, kmax=4, amp=1.0):
    """Seeded Poisson trace of scalar advection-diffusion jobs.

    Each job: arrival time (exponential gaps, mean 1/rate s), ndim 2 or 3,
    grid edge from ``edges``, RK3 step count uniform in [steps[0], steps[1]],
    storage dtype 'f32' or 'f64', velocity c ~ U[-1, 1)^ndim, viscosity nu and
    a ``modes``-mode Fourier initial condition (the mode table, not the field,
    so large grids are sampled only when admitted)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        ndim = 3 if rng.uniform() < p3d else 2
        edge = int(edges[int(rng.integers(0, len(edges)))])
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        dtype = "f32" if rng.uniform() < p_f32 else "f64"
        c = [float(v) for v in rng.uniform(-1.0, 1.0, size=ndim)]
        mt = draw_modes(rng, modes, ndim, kmax, amp)
        jobs.append(dict(id=i, arrival=t, ndim=ndim, edge=edge, steps=nsteps, dtype=dtype,
                         c=c, nu=nu, modes=mt))
    return jobs
