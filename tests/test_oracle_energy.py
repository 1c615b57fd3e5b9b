"""Pins of the oracle's energy diagnostics (1/2 sum |u|^2 and 1/2 sum |curl A|^2
with sixth-order first derivatives) against closed forms on Fourier modes:
sums of sin^2 / cos^2 over a periodic grid, the Fourier symbol of the
first-derivative stencil, and a gradient field whose discrete curl vanishes."""
import math

import numpy as np
import pytest

import oracle as O


def grid(n):
    """Coordinates 2 pi i / n_a as [z, y, x] arrays."""
    Z, Y, X = np.meshgrid(*[2 * math.pi * np.arange(v) / v for v in n[::-1]], indexing="ij")
    return X, Y, Z


def keff(k, h):
    """Symbol of the sixth-order first-derivative stencil (weights 3/4, -3/20,
    1/60 on offsets 1, 2, 3) for the mode exp(i k x): i keff."""
    return 2.0 / h * (0.75 * math.sin(k * h) - 0.15 * math.sin(2 * k * h) +
                      math.sin(3 * k * h) / 60.0)


def energies(vals, n):
    ds = [2 * math.pi / v for v in n]
    return O.energy([O.pad_periodic(v, 3) for v in vals], ds)


def test_kinetic_energy_of_a_cosine_mode_and_a_uniform_flow():
    n = (16, 12, 10)
    X, Y, Z = grid(n)
    zero = np.zeros_like(X)
    a, b = 0.7, -0.3
    vals = [zero, a * np.cos(2 * X + 0.4), np.full_like(X, b), zero] + [zero] * 4
    N = n[0] * n[1] * n[2]
    ek, em = energies(vals, n)
    assert math.isclose(ek, 0.5 * N * (a * a / 2 + b * b), rel_tol=1e-13)
    assert em == 0.0


@pytest.mark.parametrize("comp,axis", [(2, 0), (2, 1), (1, 0), (1, 2), (0, 1), (0, 2)])
def test_magnetic_energy_of_one_potential_mode(comp, axis):
    # A_comp = a cos(k x_axis): B has the single component e_comp x e_axis
    # direction with amplitude a keff, so 1/2 sum |B|^2 = a^2 keff^2 N / 4
    n = (18, 14, 12)
    X = grid(n)
    k, a = 3, 0.6
    vals = [np.zeros_like(X[0]) for _ in range(8)]
    vals[5 + comp] = a * np.cos(k * X[axis] + 0.25)
    N = n[0] * n[1] * n[2]
    h = 2 * math.pi / n[axis]
    ek, em = energies(vals, n)
    assert ek == 0.0
    assert math.isclose(em, a * a * keff(k, h) ** 2 * N / 4, rel_tol=1e-12)


def test_gradient_potential_has_no_magnetic_energy():
    # A = (c, c, c) with c = cos(x + y + z) on a cubic grid: d_y A_z = d_z A_y
    # etc. exactly (same stencil, same data), so curl A vanishes up to
    # rounding; a sign or index slip in the curl would leave ~keff^2 N
    n = (12, 12, 12)
    X, Y, Z = grid(n)
    c = np.cos(X + Y + Z)
    zero = np.zeros_like(c)
    vals = [zero, zero, zero, zero, zero, c, c, c]
    _, em = energies(vals, n)
    assert em <= 1e-24 * n[0] ** 3
    # and the same potential scaled on one component is not curl-free
    vals[7] = 2 * c
    _, em2 = energies(vals, n)
    assert em2 > 1.0


def test_superposed_modes_add_for_distinct_wavenumbers():
    # orthogonality of distinct modes over the periodic grid
    n = (20, 16, 12)
    X, Y, Z = grid(n)
    zero = np.zeros_like(X)
    vals = [zero] * 8
    vals = list(vals)
    vals[7] = 0.5 * np.cos(2 * X)            # B_y = -d_x A_z
    vals[5] = 0.3 * np.cos(3 * Y + 0.1)      # B_z = -d_y A_x
    N = n[0] * n[1] * n[2]
    want = (0.25 * keff(2, 2 * math.pi / n[0]) ** 2 + 0.09 * keff(3, 2 * math.pi / n[1]) ** 2) * N / 4
    _, em = energies(vals, n)
    assert math.isclose(em, want, rel_tol=1e-12)


def test_energy_rejects_wrong_inputs():
    with pytest.raises(ValueError):
        O.energy([np.zeros((10, 10, 10))] * 7, [1.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        O.energy([np.zeros((10, 10))] * 8, [1.0, 1.0, 1.0])
