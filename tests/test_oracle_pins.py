"""Pins of the CPU oracle against mathematics it does not encode itself.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, a transposed index or operand, a wrong coefficient) fails it:
moment conditions solved exactly, polynomial exactness, Fourier symbols on
non-cubic grids, conservation, brute-force circulant matrices, library
routines (np.pad, scipy.ndimage.correlate), the RK3 stability polynomial and
hand-derived special cases of the nonlinear right-hand side.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage

import oracle as O
from closed_forms import (W1, W2, central_weights, coords, full, kappa, lam, moments,
                          rk3_stability)

pytestmark = pytest.mark.filterwarnings("ignore")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------------------
# coefficients
# ---------------------------------------------------------------------------

def test_fd_weights_are_the_moment_solution():
    c1, c2 = O.fd_weights()
    for deriv, c in ((1, c1), (2, c2)):
        exact = central_weights(deriv, 3)
        assert [float(v) for v in exact] == list(c)
        m = moments(exact, 8)
        for k in range(7):
            assert m[k] == (math.factorial(deriv) if k == deriv else 0)
    # the leading error moment is nonzero: exactly sixth order
    assert moments(central_weights(1, 3), 7)[7] == 36
    assert moments(central_weights(2, 3), 8)[8] != 0


def butcher_from_2n(alpha, beta):
    """Butcher tableau (A, b, c) of a 2N-storage scheme w_i = alpha_i w_{i-1}
    + dt R(f_{i-1}), f_i = f_{i-1} + beta_i w_i, written as f_i = f_0 +
    sum_j A[i][j] dt R(f_j)."""
    s = len(alpha)
    # w_i = sum_j W[i][j] dt R(f_j)
    W = [[Fraction(0)] * s for _ in range(s)]
    F = [[Fraction(0)] * s for _ in range(s + 1)]  # f_i coefficients
    for i in range(s):
        for j in range(s):
            W[i][j] = (alpha[i] * W[i - 1][j] if i > 0 else 0) + (1 if j == i else 0)
        for j in range(s):
            F[i + 1][j] = F[i][j] + beta[i] * W[i][j]
    A = [F[i] for i in range(s)]
    b = F[s]
    c = [sum(row) for row in A]
    return A, b, c


def test_rk3_coefficients_are_third_order():
    al, be = O.rk3_coeffs()
    alpha = [Fraction(v).limit_denominator(1000) for v in al]
    beta = [Fraction(v).limit_denominator(1000) for v in be]
    assert [float(v) for v in alpha] == list(al) and [float(v) for v in beta] == list(be)
    assert alpha[0] == 0
    A, b, c = butcher_from_2n(alpha, beta)
    # explicit: strictly lower triangular
    assert all(A[i][j] == 0 for i in range(3) for j in range(i, 3))
    # order conditions up to three
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fraction(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fraction(1, 3)
    assert sum(b[i] * A[i][j] * c[j] for i in range(3) for j in range(3)) == Fraction(1, 6)


# ---------------------------------------------------------------------------
# padding (Eq. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,r", [((13,), 1), ((9, 7), 2), ((8, 6, 5), 3), ((5, 4, 7), 4)])
def test_periodic_fill_matches_numpy_wrap(n, r):
    inner = np.random.default_rng(1).uniform(-1, 1, tuple(reversed(n)))
    a = np.full(tuple(s + 2 * r for s in inner.shape), np.nan)
    O.interior(a, r)[...] = inner
    O.fill_periodic(a, r)
    assert np.array_equal(a, np.pad(inner, r, mode="wrap"))


# ---------------------------------------------------------------------------
# linear cross-correlation (Eq. 3, 6-7)
# ---------------------------------------------------------------------------

def circulant(n, r, g):
    """Dense matrix of the periodic cross-correlation on the interior grid,
    built by explicit modular index arithmetic (independent of any loop
    code)."""
    nd = len(n)
    N = int(np.prod(n))
    M = np.zeros((N, N))
    K = 2 * r + 1

    def lin(c):
        idx = 0
        for a in reversed(range(nd)):
            idx = idx * n[a] + c[a]
        return idx

    for p in np.ndindex(*reversed(n)):
        pc = list(reversed(p))  # (x, y, z)
        for s in np.ndindex(*([K] * nd)):
            sc = [v - r for v in reversed(s)]
            q = [(pc[a] + sc[a]) % n[a] for a in range(nd)]
            M[lin(pc), lin(q)] += g[s]
    return M


@pytest.mark.parametrize("n,r", [((13,), 3), ((9, 7), 2), ((8, 8, 8), 1), ((8, 7, 9), 3)])
def test_xcorr_brute_force_circulant(n, r):
    rng = np.random.default_rng(7)
    g = rng.uniform(-1, 1, (2 * r + 1,) * len(n))
    inner = rng.uniform(-1, 1, tuple(reversed(n)))
    out = O.interior(O.xcorr(O.pad_periodic(inner, r), r, g), r)
    ref = (circulant(n, r, g) @ inner.reshape(-1)).reshape(inner.shape)
    assert rel(out, ref) < 1e-14


@pytest.mark.parametrize("n,r", [((31,), 4), ((12, 9), 3), ((10, 9, 8), 2)])
def test_xcorr_matches_scipy_correlate_wrap(n, r):
    rng = np.random.default_rng(3)
    g = rng.uniform(-1, 1, (2 * r + 1,) * len(n))
    inner = rng.uniform(-1, 1, tuple(reversed(n)))
    out = O.interior(O.xcorr(O.pad_periodic(inner, r), r, g), r)
    ref = scipy.ndimage.correlate(inner, g, mode="wrap")
    assert rel(out, ref) < 1e-14


def test_xcorr_conservation():
    r = 3
    rng = np.random.default_rng(5)
    g = rng.uniform(-1, 1, (7, 7, 7))
    inner = rng.uniform(-1, 1, (11, 10, 9))
    out = O.interior(O.xcorr(O.pad_periodic(inner, r), r, g), r)
    assert math.fsum(out.ravel()) == pytest.approx(math.fsum(g.ravel()) * math.fsum(inner.ravel()),
                                                   rel=1e-12, abs=1e-11)


def test_three_point_smoother_on_quadratic_user_halo():
    # [1/4, 1/2, 1/4] maps x^2 to x^2 + 1/2 in grid units (halo = polynomial)
    n, r = 20, 1
    x = np.arange(-r, n + r, dtype=np.float64) - 7.0
    out = O.interior(O.xcorr(x ** 2, r, np.array([0.25, 0.5, 0.25])), r)
    assert np.array_equal(out, x[r:-r] ** 2 + 0.5)


@pytest.mark.parametrize("iters", [1, 10])
def test_three_point_smoother_fourier_closed_form(iters):
    n, k = 2 ** 10, 37
    th = 2 * math.pi * k / n
    # phase from the exact integer k*i mod n, so the sampled mode is periodic
    # to rounding of a single product (th * i itself would drift by ~1e-14)
    inner = np.cos(2 * math.pi * ((k * np.arange(n)) % n) / n + 0.3)
    res = O.interior(O.xcorr_periodic_iterate(O.pad_periodic(inner, 1), 1,
                                              np.array([0.25, 0.5, 0.25]), iters), 1)
    ref = ((1 + math.cos(th)) / 2) ** iters * inner
    assert np.max(np.abs(res - ref)) < 1e-14


def laplacian_star(r_weights):
    """3-D star tensor summing the 1-D weights along each axis."""
    c = np.array([float(v) for v in r_weights])
    r = (len(c) - 1) // 2
    g = np.zeros((2 * r + 1,) * 3)
    for a in range(3):
        idx = [r, r, r]
        for m in range(-r, r + 1):
            idx[a] = r + m
            g[tuple(idx)] += c[m + r]
    return g


def test_star_laplacian_polynomial_exactness():
    # 6th-order star Laplacian (unit spacing) is exact for degree <= 7 per axis
    r = 3
    g = laplacian_star(central_weights(2, 3))
    P = 14
    t = np.arange(P, dtype=np.float64) - 6.5
    z, y, x = np.meshgrid(t, t + 0.5, t - 1, indexing="ij")
    f = x ** 7 + 3 * y ** 6 * x + z ** 5 * y ** 2
    lap = 42 * x ** 5 + 90 * y ** 4 * x + 20 * z ** 3 * y ** 2 + 2 * z ** 5
    out = O.interior(O.xcorr(f, r, g), r)
    assert rel(out, O.interior(lap, r)) < 1e-12


def test_star_laplacian_fourier_symbol():
    n = (16, 12, 10)
    g = laplacian_star(central_weights(2, 3))
    X = coords(n)
    k = (5, -3, 4)
    inner = np.cos(k[0] * X[0] + k[1] * X[1] + k[2] * X[2] + 0.4)
    out = O.interior(O.xcorr(O.pad_periodic(inner, 3), 3, g), 3)
    # unit-spacing weights: symbol is ds^2 * lam per axis
    sym = sum(lam(k[a], n[a]) * (2 * math.pi / n[a]) ** 2 for a in range(3))
    assert rel(out, sym * inner) < 1e-13


# ---------------------------------------------------------------------------
# derivative operators
# ---------------------------------------------------------------------------

OPS = [(O.OP_X, (0,), 1), (O.OP_Y, (1,), 1), (O.OP_Z, (2,), 1), (O.OP_XX, (0,), 2),
       (O.OP_YY, (1,), 2), (O.OP_ZZ, (2,), 2), (O.OP_XY, (0, 1), 11),
       (O.OP_XZ, (0, 2), 11), (O.OP_YZ, (1, 2), 11)]


@pytest.mark.parametrize("op,axes,kind", OPS)
def test_derivative_fourier_symbols(op, axes, kind):
    n = (16, 12, 10)
    ds = [2 * math.pi / v for v in n]
    X = coords(n)
    k = (5, -3, 4)
    ph = k[0] * X[0] + k[1] * X[1] + k[2] * X[2] + 0.4
    f = O.pad_periodic(np.cos(ph), 3)
    out = O.interior(O.deriv(f, ds, op), 3)
    if kind == 1:
        ref = -kappa(k[axes[0]], n[axes[0]]) * np.sin(ph)
    elif kind == 2:
        ref = lam(k[axes[0]], n[axes[0]]) * np.cos(ph)
    else:
        ref = -kappa(k[axes[0]], n[axes[0]]) * kappa(k[axes[1]], n[axes[1]]) * np.cos(ph)
    assert rel(out, ref) < 1e-12


@pytest.mark.parametrize("op,axes,kind", OPS)
def test_derivative_polynomial_exactness(op, axes, kind):
    # user halo = the polynomial itself; exact for degree <= 6 per axis
    P = 15
    t = np.arange(P, dtype=np.float64) - 7.0
    z, y, x = np.meshgrid(t * 0.7, t * 0.9 + 0.5, t * 1.1 - 0.25, indexing="ij")
    ds = (1.1, 0.9, 0.7)
    v = [x, y, z]
    powers = (6, 5, 4)
    f = v[0] ** powers[0] * v[1] ** powers[1] * v[2] ** powers[2]

    def dpow(a, order):
        p = powers[a]
        coef = 1.0
        for i in range(order):
            coef *= p - i
        return coef * v[a] ** (p - order)

    if kind == 1:
        parts = [dpow(a, 1) if a == axes[0] else v[a] ** powers[a] for a in range(3)]
    elif kind == 2:
        parts = [dpow(a, 2) if a == axes[0] else v[a] ** powers[a] for a in range(3)]
    else:
        parts = [dpow(a, 1) if a in axes else v[a] ** powers[a] for a in range(3)]
    ref = parts[0] * parts[1] * parts[2]
    out = O.deriv(f, ds, op)
    assert rel(O.interior(out, 3), O.interior(ref, 3)) < 1e-11


def test_derivative_sixth_order_convergence():
    errs = []
    for N in (16, 32):
        n = (N, N, N)
        ds = [2 * math.pi / N] * 3
        X = coords(n)
        f = O.pad_periodic(np.sin(X[0] + 2 * X[1]) * np.cos(X[2]), 3)
        dx = np.cos(X[0] + 2 * X[1]) * np.cos(X[2])
        dxz = -np.cos(X[0] + 2 * X[1]) * np.sin(X[2])
        dyy = -4 * np.sin(X[0] + 2 * X[1]) * np.cos(X[2])
        errs.append([np.max(np.abs(O.interior(O.deriv(f, ds, op), 3) - ref))
                     for op, ref in ((O.OP_X, dx), (O.OP_XZ, dxz), (O.OP_YY, dyy))])
    for e16, e32 in zip(*errs):
        assert 50 < e16 / e32 < 80


def test_derivative_brute_force_circulant_8cubed():
    n = (8, 8, 8)
    ds = [0.5, 0.25, 2.0]
    inner = np.random.default_rng(11).uniform(-1, 1, (8, 8, 8))
    f = O.pad_periodic(inner, 3)
    for op, axes, kind in OPS:
        g = np.zeros((7, 7, 7))
        if kind == 1:
            for m in range(-3, 4):
                idx = [3, 3, 3]
                idx[2 - axes[0]] = 3 + m
                g[tuple(idx)] = W1[m + 3] / ds[axes[0]]
        elif kind == 2:
            for m in range(-3, 4):
                idx = [3, 3, 3]
                idx[2 - axes[0]] = 3 + m
                g[tuple(idx)] = W2[m + 3] / ds[axes[0]] ** 2
        else:
            for i in range(-3, 4):
                for j in range(-3, 4):
                    idx = [3, 3, 3]
                    idx[2 - axes[0]] = 3 + i
                    idx[2 - axes[1]] = 3 + j
                    g[tuple(idx)] = W1[i + 3] * W1[j + 3] / (ds[axes[0]] * ds[axes[1]])
        ref = (circulant(n, 3, g) @ inner.reshape(-1)).reshape(inner.shape)
        assert rel(O.interior(O.deriv(f, ds, op), 3), ref) < 1e-13, op


# ---------------------------------------------------------------------------
# nonlinear right-hand side: hand-derived special cases
# ---------------------------------------------------------------------------

NG = (12, 10, 14)  # non-cubic so that a transposed axis shows
NU, ETA, CS2 = 2e-3, 5e-3, 0.7  # distinct so that a swapped constant shows


def rhs_of(fields, n=NG):
    ds = [2 * math.pi / v for v in n]
    shape = tuple(reversed(n))
    padded = [O.pad_periodic(np.broadcast_to(f, shape), 3) for f in fields]
    return [O.interior(R, 3) for R in O.rhs(O.MODEL_MHD8, padded, ds, nu=NU, eta=ETA,
                                             cs2=CS2)]


def zeros8():
    return [full(NG, 0.0) for _ in range(8)]


def check(R, expect, tol=1e-12):
    scale = max(max(float(np.max(np.abs(e))) for e in expect.values() if np.ndim(e)), 1e-3)
    for k in range(8):
        e = expect.get(k, 0.0)
        err = float(np.max(np.abs(R[k] - e)))
        assert err <= tol * scale, (k, err, scale)


def test_rhs_pure_diffusion_of_lnrho_and_entropy():
    X = coords(NG)
    k = (2, -3, 1)
    ph = sum(k[a] * X[a] for a in range(3)) + 0.2
    L = 0.3 * np.cos(ph)
    f = zeros8()
    f[O.LNRHO] = L
    f[O.SS] = -L  # s + lnrho = 0: no pressure force
    lap = sum(lam(k[a], NG[a]) for a in range(3))
    check(rhs_of(f), {O.LNRHO: NU * lap * L, O.SS: -NU * lap * L})


@pytest.mark.parametrize("which", [O.LNRHO, O.SS])
def test_rhs_pressure_gradient(which):
    X = coords(NG)
    k = (1, 2, -2)
    ph = sum(k[a] * X[a] for a in range(3)) + 0.5
    f = zeros8()
    f[which] = 0.4 * np.cos(ph)
    lap = sum(lam(k[a], NG[a]) for a in range(3))
    exp = {which: NU * lap * f[which]}
    for a in range(3):
        exp[O.UX + a] = CS2 * kappa(k[a], NG[a]) * 0.4 * np.sin(ph)
    check(rhs_of(f), exp)


def test_rhs_uniform_advection_of_lnrho():
    X = coords(NG)
    U = (0.3, -0.2, 0.5)
    k = (3, 1, -2)
    ph = sum(k[a] * X[a] for a in range(3)) + 1.1
    f = zeros8()
    f[O.LNRHO] = 0.2 * np.cos(ph)
    for a in range(3):
        f[O.UX + a] = full(NG, U[a])
    kap = [kappa(k[a], NG[a]) for a in range(3)]
    lap = sum(lam(k[a], NG[a]) for a in range(3))
    exp = {O.LNRHO: sum(U[a] * kap[a] for a in range(3)) * 0.2 * np.sin(ph) + NU * lap * f[O.LNRHO]}
    for a in range(3):
        exp[O.UX + a] = CS2 * kap[a] * 0.2 * np.sin(ph)
    check(rhs_of(f), exp)


@pytest.mark.parametrize("a,b", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_rhs_shear_flow(a, b):
    # u_a = U sin(k x_b): divergence-free; viscous term and 2 nu S:S heating
    X = coords(NG)
    U, k = 0.6, 2
    f = zeros8()
    f[O.UX + a] = U * np.sin(k * X[b])
    kb, lb = kappa(k, NG[b]), lam(k, NG[b])
    exp = {O.UX + a: NU * lb * U * np.sin(k * X[b]),
           O.SS: NU * kb ** 2 * U ** 2 * np.cos(k * X[b]) ** 2}
    check(rhs_of(f), exp)


@pytest.mark.parametrize("a", [0, 1, 2])
def test_rhs_compressive_flow(a):
    # u_a = U sin(k x_a): div u, self-advection, 4/3 nu viscous and S:S terms
    X = coords(NG)
    U, k = 0.5, 3
    f = zeros8()
    s, c = np.sin(k * X[a]), np.cos(k * X[a])
    f[O.UX + a] = U * s
    ka, la = kappa(k, NG[a]), lam(k, NG[a])
    exp = {O.LNRHO: -ka * U * c,
           O.UX + a: -ka * U * U * s * c + NU * (4.0 / 3.0) * la * U * s,
           O.SS: (4.0 / 3.0) * NU * ka ** 2 * U ** 2 * c ** 2}
    check(rhs_of(f), exp)


def test_rhs_grad_div_mixed_term():
    # u_y = U sin(kx x + ky y): grad(div u) needs the mixed derivative d_x d_y
    X = coords(NG)
    U, kx, ky = 0.4, 2, 3
    th = kx * X[0] + ky * X[1]
    s, c = np.sin(th), np.cos(th)
    f = zeros8()
    f[O.UY] = U * s
    Kx, Ky = kappa(kx, NG[0]), kappa(ky, NG[1])
    Lx, Ly = lam(kx, NG[0]), lam(ky, NG[1])
    exp = {O.LNRHO: -Ky * U * c,
           O.UX: -(NU / 3.0) * Kx * Ky * U * s,
           O.UY: -U * s * Ky * U * c + NU * ((Lx + Ly) + Ly / 3.0) * U * s,
           O.SS: 2 * NU * ((2.0 / 3.0) * Ky ** 2 + 0.5 * Kx ** 2) * U ** 2 * c ** 2}
    check(rhs_of(f), exp)


def test_rhs_magnetic_tension_and_induction():
    # A_z = a sin(k x), plus a uniform flow along x for the u x B term
    X = coords(NG)
    a, k, U = 0.3, 2, 0.7
    s, c = np.sin(k * X[0]), np.cos(k * X[0])
    K, L = kappa(k, NG[0]), lam(k, NG[0])
    f = zeros8()
    f[O.AZ] = a * s
    # B = (0, -K a cos, 0); j = (0, 0, -L a sin); j x B = (-L K a^2 sin cos, 0, 0)
    check(rhs_of(f), {O.UX: -L * K * a * a * s * c, O.SS: ETA * L * L * a * a * s * s,
                      O.AZ: ETA * L * a * s})
    f[O.UX] = full(NG, U)
    # u x B = (0, 0, U B_y)
    check(rhs_of(f), {O.UX: -L * K * a * a * s * c, O.SS: ETA * L * L * a * a * s * s,
                      O.AZ: -U * K * a * c + ETA * L * a * s})


def test_rhs_current_mixed_term():
    # A_y = a sin(kx x + ky y): j needs grad(div A) with the mixed d_x d_y
    X = coords(NG)
    a, kx, ky = 0.25, 1, 2
    th = kx * X[0] + ky * X[1]
    s, c = np.sin(th), np.cos(th)
    Kx, Ky = kappa(kx, NG[0]), kappa(ky, NG[1])
    Lx, Ly = lam(kx, NG[0]), lam(ky, NG[1])
    f = zeros8()
    f[O.AY] = a * s
    # B = (0, 0, Kx a cos); j = (-Kx Ky a sin, -Lx a sin, 0)
    exp = {O.UX: -Lx * Kx * a * a * s * c, O.UY: Kx * Kx * Ky * a * a * s * c,
           O.SS: ETA * (Kx ** 2 * Ky ** 2 + Lx ** 2) * a * a * s * s,
           O.AY: ETA * (Lx + Ly) * a * s}
    check(rhs_of(f), exp)


def test_rhs_shear_times_density_gradient():
    # 2 nu S.grad(lnrho) with u_x = U sin(k y) and lnrho = L sin(q x)
    X = coords(NG)
    U, L, k, q = 0.5, 0.2, 2, 3
    f = zeros8()
    f[O.UX] = U * np.sin(k * X[1])
    f[O.LNRHO] = L * np.sin(q * X[0])
    Ky, Ly = kappa(k, NG[1]), lam(k, NG[1])
    Kx, Lx = kappa(q, NG[0]), lam(q, NG[0])
    cy, cx = np.cos(k * X[1]), np.cos(q * X[0])
    exp = {O.LNRHO: -U * np.sin(k * X[1]) * Kx * L * cx + NU * Lx * f[O.LNRHO],
           O.UX: -CS2 * Kx * L * cx + NU * Ly * f[O.UX],
           O.UY: NU * Ky * Kx * U * L * cy * cx,
           O.SS: NU * Ky ** 2 * U ** 2 * cy ** 2}
    check(rhs_of(f), exp)


def test_rhs_force_free_abc_field():
    # ABC potential: curl A = kappa A, div A = 0, so j x B = 0 and u = 0
    n = (16, 16, 16)
    X = coords(n)
    k = 2
    A_, B_, C_ = 0.3, 0.2, 0.1
    f = [full(n, 0.0) for _ in range(8)]
    f[O.AX] = A_ * np.sin(k * X[2]) + C_ * np.cos(k * X[1])
    f[O.AY] = B_ * np.sin(k * X[0]) + A_ * np.cos(k * X[2])
    f[O.AZ] = C_ * np.sin(k * X[1]) + B_ * np.cos(k * X[0])
    L = lam(k, 16)
    A2 = f[O.AX] ** 2 + f[O.AY] ** 2 + f[O.AZ] ** 2
    exp = {O.SS: ETA * L * L * A2, O.AX: ETA * L * f[O.AX], O.AY: ETA * L * f[O.AY],
           O.AZ: ETA * L * f[O.AZ]}
    check(rhs_of(f, n), exp)


# ---------------------------------------------------------------------------
# RK3 substeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_rk3_advdiff_stability_polynomial(ndim):
    n = (16, 12, 10)[:ndim]
    ds = [2 * math.pi / v for v in n]
    X = coords(n)
    k = (3, -2, 1)[:ndim]
    c = (0.7, -0.4, 0.3)[:ndim]
    nu = 0.05
    ph = sum(k[a] * X[a] for a in range(ndim)) + 0.3
    dt = 0.1 * min(ds)
    f0 = np.cos(ph)
    out = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 1, nu=nu, c=c)[0]
    # symbol of R on exp(i k.x): -i c.kappa + nu sum lam
    sym = complex(nu * sum(lam(k[a], n[a]) for a in range(ndim)),
                  -sum(c[a] * kappa(k[a], n[a]) for a in range(ndim)))
    G = rk3_stability(dt * sym)
    ref = np.real(G * np.exp(1j * ph))
    assert np.max(np.abs(O.interior(out, 3) - ref)) < 1e-14
    # several steps compound
    out5 = O.rk3_steps(O.MODEL_ADVDIFF, [O.pad_periodic(f0, 3)], ds, dt, 5, nu=nu, c=c)[0]
    assert np.max(np.abs(O.interior(out5, 3) - np.real(G ** 5 * np.exp(1j * ph)))) < 1e-13


def test_rk3_mhd8_diffusive_special_case():
    # u = A = 0, s = -lnrho: both scalars diffuse; per-mode amplification is
    # the RK3 stability polynomial of dt nu lam
    X = coords(NG)
    k = (1, -2, 3)
    ph = sum(k[a] * X[a] for a in range(3)) + 0.9
    f = zeros8()
    f[O.LNRHO] = 0.3 * np.cos(ph)
    f[O.SS] = -0.3 * np.cos(ph)
    ds = [2 * math.pi / v for v in NG]
    dt = 0.1 * min(ds)
    f = [np.broadcast_to(v, tuple(reversed(NG))) for v in f]
    out = O.rk3_steps(O.MODEL_MHD8, [O.pad_periodic(v, 3) for v in f], ds, dt, 2,
                      nu=0.05, eta=ETA, cs2=CS2)
    G = rk3_stability(dt * 0.05 * sum(lam(k[a], NG[a]) for a in range(3)))
    assert np.max(np.abs(O.interior(out[O.LNRHO], 3) - G ** 2 * f[O.LNRHO])) < 1e-14
    assert np.max(np.abs(O.interior(out[O.SS], 3) - G ** 2 * f[O.SS])) < 1e-14
    for q in (O.UX, O.UY, O.UZ, O.AX, O.AY, O.AZ):
        assert np.max(np.abs(O.interior(out[q], 3))) < 1e-15


def test_rk3_substep_at_matches_full_grid():
    n = (10, 9, 8)
    ds = [2 * math.pi / v for v in n]
    rng = np.random.default_rng(4)
    fin = [O.pad_periodic(rng.uniform(-0.01, 0.01, tuple(reversed(n))), 3) for _ in range(8)]
    w = [rng.uniform(-1e-3, 1e-3, fin[0].shape) for _ in range(8)]
    pts = np.array([[0, 0, 0], [9, 8, 7], [4, 3, 5], [1, 8, 0]])
    w_in = np.array([[w[k][p[2] + 3, p[1] + 3, p[0] + 3] for p in pts] for k in range(8)])
    wf = [a.copy() for a in w]
    fout = O.rk3_substep(O.MODEL_MHD8, 1, fin, wf, ds, 0.01)
    w_at, f_at = O.rk3_substep_at(O.MODEL_MHD8, 1, fin, w_in, ds, 0.01, pts)
    for k in range(8):
        for i, p in enumerate(pts):
            assert w_at[k, i] == wf[k][p[2] + 3, p[1] + 3, p[0] + 3]
            assert f_at[k, i] == fout[k][p[2] + 3, p[1] + 3, p[0] + 3]
    # fout's halo is periodic
    for k in range(8):
        assert np.array_equal(fout[k], np.pad(O.interior(fout[k], 3), 3, mode="wrap"))


def test_xcorr_at_matches_full_grid():
    rng = np.random.default_rng(9)
    g = rng.uniform(-1, 1, (7, 7, 7))
    a = O.pad_periodic(rng.uniform(-1, 1, (9, 8, 10)), 3)
    full_out = O.xcorr(a, 3, g)
    pts = np.array([[0, 0, 0], [9, 7, 8], [5, 2, 3]])
    at = O.xcorr_at(a, 3, g, pts)
    for i, p in enumerate(pts):
        assert at[i] == full_out[p[2] + 3, p[1] + 3, p[0] + 3]


# ---------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------

def test_reduce_matches_exact_sums():
    rng = np.random.default_rng(2)
    inner = rng.uniform(-1, 1, (13, 11, 9))
    a = O.pad_periodic(inner, 3)
    a[0, 0, 0] = 1e6  # halo must not count
    s, s2, mx = O.reduce(a, 3)
    assert s == pytest.approx(math.fsum(inner.ravel()), rel=1e-13, abs=1e-12)
    assert s2 == pytest.approx(math.fsum((inner ** 2).ravel()), rel=1e-13)
    assert mx == np.max(np.abs(inner))
