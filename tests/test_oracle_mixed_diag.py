"""Pins of the oracle's diagonal mixed derivative (12 taps on the two
diagonals of a coordinate plane) and of the MHD banks that use it: exact
derivatives of polynomials up to total degree 7 (and not 8: order exactly 6),
sixth-order convergence on smooth periodic fields, the tap footprint, and the
right-hand sides, which must equal the tensor-product form wherever no mixed
term is active and converge to the continuous equations either way."""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_mhd_full import (CS02, ETA, MHD, NU, continuous_rhs, field_and_derivs,
                                  modes)

PLANES = [(O.OP_XY_DIAG, 0, 1), (O.OP_XZ_DIAG, 0, 2), (O.OP_YZ_DIAG, 1, 2)]


def coords(n, ds):
    """Padded coordinates x_a = (i - 3) ds_a as [z, y, x] arrays (not periodic:
    the padding holds the polynomial's own values)."""
    ax = [(np.arange(v + 6) - 3) * h for v, h in zip(n, ds)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


@pytest.mark.parametrize("op,a,b", PLANES)
def test_exact_on_polynomials_up_to_degree_seven(op, a, b):
    n, ds = (9, 8, 7), (0.3, 0.25, 0.2)
    X = coords(n, ds)
    for i in range(1, 7):
        for j in range(1, 8 - i):  # i + j <= 7
            f = X[a] ** i * X[b] ** j * (1.0 + 0.5 * X[3 - a - b])  # third axis factor
            want = i * j * X[a] ** (i - 1) * X[b] ** (j - 1) * (1.0 + 0.5 * X[3 - a - b])
            got = O.interior(O.deriv(f, ds, op), 3)
            assert np.allclose(got, O.interior(want, 3), rtol=1e-9, atol=1e-9), (i, j)


@pytest.mark.parametrize("op,a,b", PLANES)
def test_not_exact_at_degree_eight(op, a, b):
    n, ds = (9, 8, 7), (0.3, 0.25, 0.2)
    X = coords(n, ds)
    # the diagonal lines carry s^8 coefficients h_a^i h_b^j and
    # h_a^i (-h_b)^j, so their leading errors cancel for even j: take j odd
    f = X[a] ** 3 * X[b] ** 5
    want = 15 * X[a] ** 2 * X[b] ** 4
    err = np.max(np.abs(O.interior(O.deriv(f, ds, op), 3) - O.interior(want, 3)))
    assert err > 1e-6


def test_twelve_taps_on_the_diagonals():
    n, ds = (13, 13, 13), (1.0, 1.0, 1.0)
    imp = np.zeros((19, 19, 19))
    imp[9, 9, 9] = 1.0  # [z, y, x] padded coordinates of the interior centre
    for op, a, b in PLANES:
        resp = O.deriv(imp, ds, op)
        nz = np.argwhere(resp != 0.0) - 9  # offsets (z, y, x) of points that see the impulse
        assert len(nz) == 12
        for off in nz:
            o = off[::-1]  # (x, y, z)
            c = 3 - a - b
            assert o[c] == 0 and abs(o[a]) == abs(o[b]) and 1 <= abs(o[a]) <= 3
        # the weights of one diagonal pair sum to zero against the other
        assert abs(resp.sum()) < 1e-15


def test_sixth_order_convergence_on_a_periodic_field():
    errs = []
    for n in ((16, 16, 16), (32, 32, 32)):
        ds = [2 * math.pi / v for v in n]
        f, g, h = field_and_derivs(n, modes(5, count=4, kmax=2))
        pad = O.pad_periodic(f, 3)
        e = []
        for op, a, b in PLANES:
            got = O.interior(O.deriv(pad, ds, op), 3)
            e.append(np.max(np.abs(got - h[a][b])) / np.max(np.abs(h[a][b])))
        errs.append(e)
    ratio = np.array(errs[0]) / np.array(errs[1])
    # 2^6 = 64 asymptotically; fifth order would give 32, eighth 256
    assert np.all(ratio > 40) and np.all(ratio < 80), ratio


@pytest.mark.parametrize("model", [O.MODEL_MHD8, O.MODEL_MHD_FULL])
def test_rhs_equals_tensor_form_when_no_mixed_term_is_active(model):
    # every vector component depends on its own coordinate only, so each
    # d_a d_b v_b with a != b vanishes in both forms (exactly on the
    # diagonals, to rounding in the tensor product's 49-term sum); everything
    # else is the same arithmetic
    n = (12, 10, 8)
    ds = [2 * math.pi / v for v in n]
    Z, Y, X = np.meshgrid(*[2 * math.pi * np.arange(v) / v for v in n[::-1]], indexing="ij")
    own = [np.sin(X + 0.3), np.cos(2 * Y), np.sin(Z - 0.2)]
    vals = [0.1 * np.sin(X + Y), 0.2 * own[0], 0.1 * own[1], 0.3 * own[2],
            0.1 * np.cos(Y - Z), 0.2 * own[0], 0.3 * own[1], 0.1 * own[2]]
    pads = [O.pad_periodic(v, 3) for v in vals]
    kw = dict(nu=NU, eta=ETA, cs2=CS02, mhd=MHD if model == O.MODEL_MHD_FULL else None)
    R_t = O.rhs(model, pads, ds, **kw)
    R_d = O.rhs(model, pads, ds, mixed=O.MIXED_DIAG, **kw)
    for k in range(8):
        scale = max(np.max(np.abs(R_t[k])), 1e-300)
        assert np.max(np.abs(R_t[k] - R_d[k])) <= 1e-14 * scale, k


def test_full_rhs_with_diagonal_mixed_terms_converges_at_sixth_order():
    fm = [modes(10 + k) for k in range(8)]
    errs = []
    for n in ((20, 18, 16), (40, 36, 32)):
        want, vals = continuous_rhs(n, fm, NU, ETA, CS02, MHD)
        ds = [2 * math.pi / v for v in n]
        pads = [O.pad_periodic(v, 3) for v in vals]
        got = O.rhs(O.MODEL_MHD_FULL, pads, ds, nu=NU, eta=ETA, cs2=CS02, mhd=MHD,
                    mixed=O.MIXED_DIAG)
        errs.append([np.max(np.abs(O.interior(got[k], 3) - want[k])) / np.max(np.abs(want[k]))
                     for k in range(8)])
    ratio = np.array(errs[0]) / np.array(errs[1])
    assert np.all(ratio > 40), ratio


def test_diagonal_and_tensor_banks_differ_only_at_sixth_order():
    # a velocity with mixed terms: the two forms differ, by O(h^6)
    diffs = []
    for n in ((16, 16, 16), (32, 32, 32)):
        ds = [2 * math.pi / v for v in n]
        Z, Y, X = np.meshgrid(*[2 * math.pi * np.arange(v) / v for v in n[::-1]],
                              indexing="ij")
        uy = 0.2 * np.sin(X + 2 * Y + 0.1)
        zero = np.zeros_like(uy)
        vals = [zero, zero, uy, zero, zero, zero, zero, zero]
        pads = [O.pad_periodic(v, 3) for v in vals]
        R_t = O.rhs(O.MODEL_MHD8, pads, ds, nu=NU, eta=ETA, cs2=CS02)
        R_d = O.rhs(O.MODEL_MHD8, pads, ds, nu=NU, eta=ETA, cs2=CS02, mixed=O.MIXED_DIAG)
        d = O.interior(R_d[1] - R_t[1], 3)  # nu/3 d_x d_y u_y in R_ux
        assert np.max(np.abs(d)) > 0
        diffs.append(np.max(np.abs(d)))
    assert 40 < diffs[0] / diffs[1] < 80, diffs


def test_mixed_mode_is_rejected_for_the_scalar_model():
    with pytest.raises(ValueError):
        O.rhs(O.MODEL_ADVDIFF, [np.zeros((10, 10, 10))], [1.0, 1.0, 1.0], mixed=O.MIXED_DIAG)
    with pytest.raises(ValueError):
        O.rhs(O.MODEL_MHD8, [np.zeros((10, 10, 10))] * 8, [1.0, 1.0, 1.0], mixed="box")
