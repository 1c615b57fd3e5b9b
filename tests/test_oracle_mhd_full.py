"""Pins of the oracle's full non-ideal MHD right-hand side (Eq. A1-A4 with an
ideal-gas closure) against an independent NumPy evaluation of the same
equations from exact derivatives of smooth Fourier fields (the discrete
right-hand side must converge to it at sixth order), with lap T taken by
spectral differentiation of T itself, and against closed-form special cases."""
import math

import numpy as np
import pytest

import oracle as O

MHD = dict(zeta=3e-3, mu0=1.3, gamma=5.0 / 3.0, cp=1.7, lnrho0=0.2, K=4e-3, heat=2e-3,
           cool=5e-4)
NU, ETA, CS02 = 2e-3, 3e-3, 0.8


def modes(seed, count=3, kmax=2, amp=0.15):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = rng.integers(-kmax, kmax + 1, 3)
        if not k.any():
            k[0] = 1
        out.append((k, rng.uniform(-amp, amp), rng.uniform(0, 2 * math.pi)))
    return out


def field_and_derivs(n, mode_list):
    """Value, gradient [a] and Hessian [a][b] of sum a cos(k.x + phi) on the
    grid x_a = 2 pi i / n_a, arrays in [z, y, x] order."""
    X = np.meshgrid(*[2 * math.pi * np.arange(v) / v for v in n], indexing="ij")  # x, y, z
    X = [np.transpose(c, (2, 1, 0)) for c in X]
    val = np.zeros(X[0].shape)
    grad = [np.zeros_like(val) for _ in range(3)]
    hess = [[np.zeros_like(val) for _ in range(3)] for _ in range(3)]
    for k, a, ph in mode_list:
        arg = ph + sum(k[d] * X[d] for d in range(3))
        c, s = np.cos(arg), np.sin(arg)
        val += a * c
        for p in range(3):
            grad[p] += -a * k[p] * s
            for q in range(3):
                hess[p][q] += -a * k[p] * k[q] * c
    return val, grad, hess


def spectral_laplacian(f):
    n = f.shape
    k = [np.fft.fftfreq(m, d=1.0 / m) for m in n]  # integer wavenumbers, period 2 pi
    KZ, KY, KX = np.meshgrid(*k, indexing="ij")
    return np.real(np.fft.ifftn(-(KX ** 2 + KY ** 2 + KZ ** 2) * np.fft.fftn(f)))


def continuous_rhs(n, fields_modes, nu, eta, cs02, m):
    """A1-A4 evaluated from exact derivatives (written independently of the
    oracle); returns the 8 right-hand sides on the grid."""
    F = [field_and_derivs(n, fm) for fm in fields_modes]
    l, gl, hl = F[0]
    s, gs, hs = F[4]
    u = [F[1 + b][0] for b in range(3)]
    du = [[F[1 + b][1][a] for b in range(3)] for a in range(3)]       # du[a][b] = d_a u_b
    dA = [[F[5 + b][1][a] for b in range(3)] for a in range(3)]
    lap = lambda h: h[0][0] + h[1][1] + h[2][2]
    lapu = [lap(F[1 + b][2]) for b in range(3)]
    lapA = [lap(F[5 + b][2]) for b in range(3)]
    gdivu = [sum(F[1 + b][2][a][b] for b in range(3)) for a in range(3)]
    gdivA = [sum(F[5 + b][2][a][b] for b in range(3)) for a in range(3)]
    divu = du[0][0] + du[1][1] + du[2][2]
    B = [dA[1][2] - dA[2][1], dA[2][0] - dA[0][2], dA[0][1] - dA[1][0]]
    j = [(gdivA[a] - lapA[a]) / m["mu0"] for a in range(3)]
    rho = np.exp(l)
    g, cp = m["gamma"], m["cp"]
    cs2 = cs02 * np.exp(g * s / cp + (g - 1) * (l - m["lnrho0"]))
    T = cs2 / ((g - 1) * cp)
    lapT = spectral_laplacian(T)  # independent of the chain rule the oracle uses
    S = [[0.5 * (du[a][b] + du[b][a]) - (divu / 3 if a == b else 0) for b in range(3)]
         for a in range(3)]
    cross = lambda p, q: [p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2],
                          p[0] * q[1] - p[1] * q[0]]
    jxB, uxB = cross(j, B), cross(u, B)
    R = [None] * 8
    R[0] = -sum(u[a] * gl[a] for a in range(3)) - divu
    for a in range(3):
        adv = sum(u[b] * du[b][a] for b in range(3))
        Sgl = sum(S[a][b] * gl[b] for b in range(3))
        R[1 + a] = (-adv - cs2 * (gs[a] / cp + gl[a]) + jxB[a] / rho +
                    nu * (lapu[a] + gdivu[a] / 3 + 2 * Sgl) + m["zeta"] * gdivu[a])
    SS = sum(S[a][b] ** 2 for a in range(3) for b in range(3))
    jj = sum(j[a] ** 2 for a in range(3))
    R[4] = (-sum(u[a] * gs[a] for a in range(3)) +
            (m["heat"] - m["cool"] + m["K"] * lapT + eta * m["mu0"] * jj + 2 * rho * nu * SS +
             m["zeta"] * rho * divu ** 2) / (rho * T))
    for a in range(3):
        R[5 + a] = uxB[a] + eta * lapA[a]
    return R, [f[0] for f in F]


def oracle_rhs_full(n, vals):
    ds = [2 * math.pi / v for v in n]
    pads = [O.pad_periodic(v, 3) for v in vals]
    R = O.rhs(O.MODEL_MHD_FULL, pads, ds, nu=NU, eta=ETA, cs2=CS02, mhd=MHD)
    return [O.interior(r, 3) for r in R]


def test_full_rhs_converges_at_sixth_order_to_the_continuous_equations():
    fm = [modes(10 + k) for k in range(8)]
    errs = []
    for n in ((20, 18, 16), (40, 36, 32)):
        want, vals = continuous_rhs(n, fm, NU, ETA, CS02, MHD)
        got = oracle_rhs_full(n, vals)
        errs.append([np.max(np.abs(got[k] - want[k])) / np.max(np.abs(want[k])) for k in range(8)])
    e1, e2 = np.array(errs[0]), np.array(errs[1])
    assert np.all(e2 < 5e-5), e2
    # halving the spacing divides the error by 2^6 = 64 (allow 40 for the
    # pre-asymptotic regime)
    assert np.all(e1 / e2 > 40), e1 / e2


def test_uniform_state_gives_only_the_heating_balance():
    n = (8, 7, 6)
    vals = [np.full(n[::-1], v) for v in (0.3, 0.1, -0.2, 0.05, 0.4, 0.7, -0.1, 0.2)]
    R = oracle_rhs_full(n, vals)
    g, cp = MHD["gamma"], MHD["cp"]
    rho = math.exp(0.3)
    cs2 = CS02 * math.exp(g * 0.4 / cp + (g - 1) * (0.3 - MHD["lnrho0"]))
    T = cs2 / ((g - 1) * cp)
    for k in (0, 1, 2, 3, 5, 6, 7):
        assert np.max(np.abs(R[k])) <= 1e-15, k
    assert np.allclose(R[4], (MHD["heat"] - MHD["cool"]) / (rho * T), rtol=1e-14, atol=0)


def test_lorentz_force_scales_with_inverse_density():
    # u = 0, s constant, lnrho constant: R_u is j x B / rho alone
    n = (24, 20, 22)
    fm = [modes(30 + k) for k in range(3)]
    A = [field_and_derivs(n, f)[0] for f in fm]
    zero = np.zeros(n[::-1])
    out = []
    for c in (0.0, 0.7):
        vals = [np.full(n[::-1], c), zero, zero, zero, np.full(n[::-1], 0.25)] + A
        out.append(oracle_rhs_full(n, vals))
    for a in range(3):
        assert np.max(np.abs(out[0][1 + a])) > 1e-4
        assert np.allclose(out[1][1 + a], out[0][1 + a] * math.exp(-0.7), rtol=1e-12, atol=1e-15)


def test_pressure_force_uses_the_ideal_gas_sound_speed():
    n = (24, 10, 12)
    ds = [2 * math.pi / v for v in n]
    l = field_and_derivs(n, [(np.array([1, 0, 0]), 0.3, 0.4), (np.array([2, 1, 0]), 0.1, 1.0)])[0]
    zero = np.zeros(n[::-1])
    vals = [l, zero, zero, zero, np.full(n[::-1], -0.3), zero, zero, zero]
    R = oracle_rhs_full(n, vals)
    g, cp = MHD["gamma"], MHD["cp"]
    cs2 = CS02 * np.exp(g * -0.3 / cp + (g - 1) * (l - MHD["lnrho0"]))
    pad = O.pad_periodic(l, 3)
    for a in range(3):
        dl = O.interior(O.deriv(pad, ds, a), 3)
        assert np.allclose(R[1 + a], -cs2 * dl, rtol=1e-12, atol=1e-15)


def test_bulk_viscosity_terms():
    # compressive flow u = (a sin x, 0, 0): the zeta terms are zeta grad(div u)
    # in R_u and zeta rho (div u)^2 / (rho T) in R_s
    n = (32, 6, 6)
    ds = [2 * math.pi / v for v in n]
    ux = field_and_derivs(n, [(np.array([1, 0, 0]), 0.2, 0.0)])[0]
    zero = np.zeros(n[::-1])
    base = [np.full(n[::-1], 0.1), ux, zero, zero, np.full(n[::-1], 0.2), zero, zero, zero]
    pads = [O.pad_periodic(v, 3) for v in base]
    R1 = O.rhs(O.MODEL_MHD_FULL, pads, ds, nu=NU, eta=ETA, cs2=CS02, mhd=MHD)
    R0 = O.rhs(O.MODEL_MHD_FULL, pads, ds, nu=NU, eta=ETA, cs2=CS02, mhd=dict(MHD, zeta=0.0))
    divu = O.interior(O.deriv(pads[1], ds, 0), 3)
    gdivu = O.interior(O.deriv(pads[1], ds, 3), 3)  # d_xx u_x
    g, cp = MHD["gamma"], MHD["cp"]
    rho = math.exp(0.1)
    T = CS02 * math.exp(g * 0.2 / cp + (g - 1) * (0.1 - MHD["lnrho0"])) / ((g - 1) * cp)
    d_u = O.interior(R1[1] - R0[1], 3)
    d_s = O.interior(R1[4] - R0[4], 3)
    assert np.allclose(d_u, MHD["zeta"] * gdivu, rtol=1e-9, atol=1e-16)
    assert np.allclose(d_s, MHD["zeta"] * rho * divu ** 2 / (rho * T), rtol=1e-9, atol=1e-16)


def test_rk_substep_of_the_full_model_runs_and_matches_its_rhs():
    n = (10, 9, 8)
    fm = [modes(50 + k) for k in range(8)]
    vals = [field_and_derivs(n, f)[0] for f in fm]
    pads = [O.pad_periodic(v, 3) for v in vals]
    ds = [2 * math.pi / v for v in n]
    dt = 1e-3
    w = [np.zeros_like(p) for p in pads]
    out = O.rk3_substep(O.MODEL_MHD_FULL, 0, pads, w, ds, dt, nu=NU, eta=ETA, cs2=CS02, mhd=MHD)
    R = O.rhs(O.MODEL_MHD_FULL, pads, ds, nu=NU, eta=ETA, cs2=CS02, mhd=MHD)
    for k in range(8):
        # stage 0: w = dt R, f' = f + beta_0 w (beta_0 = 1/3)
        assert np.allclose(O.interior(w[k], 3), dt * O.interior(R[k], 3), rtol=1e-14, atol=0)
        assert np.allclose(O.interior(out[k], 3), vals[k] + (dt / 3) * O.interior(R[k], 3),
                           rtol=1e-14, atol=1e-17)
