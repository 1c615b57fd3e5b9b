"""Python view of the plain FP64 CPU oracle (oracle/stencil_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package. It shares no
code with the GPU path.

Arrays are NumPy float64, C-contiguous, padded by r cells on every active axis
(paper Eq. 2, Fig. 1) and indexed [z, y, x] in NumPy order so that x is the
fastest axis (row-wise scan order, Sec. 4.4). ``n`` tuples are (nx, ny, nz).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MODEL_MHD8 = 0
MODEL_ADVDIFF = 1
MODEL_MHD_FULL = 2
# constants of the full model that the paper leaves to its reference [44]
# (ideal-gas closure; heating, cooling, conduction, bulk viscosity)
MHD_DEFAULTS = dict(zeta=0.0, mu0=1.0, gamma=5.0 / 3.0, cp=1.0, lnrho0=0.0, K=0.0, heat=0.0,
                    cool=0.0)
# field order of the 8-field system (Table A1)
LNRHO, UX, UY, UZ, SS, AX, AY, AZ = range(8)
# window filter codes (max filter of Sec. 2.3; median filter of Sec. 1)
FILTER_MAX, FILTER_MIN, FILTER_MEDIAN = 1, 2, 3
# derivative operator codes
OP_X, OP_Y, OP_Z, OP_XX, OP_YY, OP_ZZ, OP_XY, OP_XZ, OP_YZ = range(9)
# mixed derivatives from the diagonals of the plane (12 taps)
OP_XY_DIAG, OP_XZ_DIAG, OP_YZ_DIAG = 9, 10, 11
# mixed-derivative forms of the MHD derivative bank
MIXED_TENSOR, MIXED_DIAG = "tensor", "diag"

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def lib():
    """Load liboracle.so, building it with gcc first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_fill_periodic.argtypes = [_dp, ctypes.c_int, _lp, ctypes.c_int]
        L.oracle_xcorr.argtypes = [_dp, _dp, ctypes.c_int, _lp, ctypes.c_int, _dp]
        L.oracle_xcorr_at.argtypes = [_dp, ctypes.c_int, _lp, ctypes.c_int, _dp, _lp,
                                      ctypes.c_long, _dp]
        L.oracle_fd_weights.argtypes = [_dp, _dp]
        L.oracle_deriv.argtypes = [_dp, _dp, ctypes.c_int, _lp, _dp, ctypes.c_int]
        L.oracle_deriv.restype = ctypes.c_int
        L.oracle_rhs.argtypes = [ctypes.c_int, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                 ctypes.c_int, _lp, _dp, _dp]
        L.oracle_rhs.restype = ctypes.c_int
        L.oracle_rk3_coeffs.argtypes = [_dp, _dp]
        L.oracle_rk3_substep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_dp),
                                         ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                         ctypes.c_int, _lp, _dp, _dp, ctypes.c_double]
        L.oracle_rk3_substep.restype = ctypes.c_int
        L.oracle_rk3_substep_at.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_dp),
                                            _dp, ctypes.c_int, _lp, _dp, _dp,
                                            ctypes.c_double, _lp, ctypes.c_long, _dp, _dp]
        L.oracle_rk3_substep_at.restype = ctypes.c_int
        L.oracle_reduce.argtypes = [_dp, ctypes.c_int, _lp, ctypes.c_int, _dp]
        L.oracle_energy.argtypes = [ctypes.POINTER(_dp), _lp, _dp, _dp]
        L.oracle_filter.argtypes = [_dp, _dp, ctypes.c_int, _lp, ctypes.c_int, _dp, ctypes.c_int]
        L.oracle_filter_at.argtypes = [_dp, ctypes.c_int, _lp, ctypes.c_int, _dp, ctypes.c_int,
                                       _lp, ctypes.c_long, _dp]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need C-contiguous float64"
    return a.ctypes.data_as(_dp)


def _dims(a, r):
    """(ndim, n as ctypes long[3]) from a padded array."""
    nd = a.ndim
    n = [a.shape[nd - 1 - k] - 2 * r for k in range(nd)] + [1] * (3 - nd)
    if min(n[:nd]) < 1:
        raise ValueError("array smaller than its padding")
    return nd, (ctypes.c_long * 3)(*n)


def _ptrs(arrs):
    if any(a.shape != arrs[0].shape for a in arrs):
        raise ValueError("all fields must have the same padded shape")
    return (_dp * len(arrs))(*[_ptr(a) for a in arrs])


def _d3(v):
    v = list(v) + [0.0] * (3 - len(v))
    return (ctypes.c_double * 3)(*v)


# --------------------------------------------------------------------------
# padding psi (Eq. 2)
# --------------------------------------------------------------------------

def padded_shape(n, r):
    """NumPy shape of a field with interior n = (nx[, ny[, nz]]) padded by r."""
    return tuple(int(n[k]) + 2 * r for k in reversed(range(len(n))))


def interior(a, r):
    return a[tuple(slice(r, s - r) for s in a.shape)]


def fill_periodic(a, r):
    """Periodic boundary function: fill the halo of padded array a in place."""
    nd, n = _dims(a, r)
    lib().oracle_fill_periodic(_ptr(a), nd, n, r)
    return a


def pad_periodic(inner, r):
    """New padded array whose interior is ``inner`` and halo is periodic."""
    inner = np.asarray(inner, dtype=np.float64)
    a = np.zeros(tuple(s + 2 * r for s in inner.shape))
    interior(a, r)[...] = inner
    return fill_periodic(a, r)


# --------------------------------------------------------------------------
# linear cross-correlation (Eq. 3, Eq. 6-7)
# --------------------------------------------------------------------------

def xcorr(a, r, g):
    """Cross-correlation of padded a with the dense (2r+1)^ndim tensor g
    (NumPy order [sz, sy, sx]). Returns a padded array, halo zero."""
    nd, n = _dims(a, r)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (2 * r + 1,) * nd
    out = np.zeros_like(a)
    lib().oracle_xcorr(_ptr(a), _ptr(out), nd, n, r, _ptr(g))
    return out


def xcorr_periodic_iterate(a, r, g, iters):
    """``iters`` chained applications with a periodic halo refresh before
    each one; the input is not modified. Returns the padded result."""
    cur = fill_periodic(a.copy(), r)
    for _ in range(iters):
        cur = fill_periodic(xcorr(cur, r, g), r)
    return cur


def filter(a, r, mask, op):
    """Window filter of padded a (op FILTER_MAX / FILTER_MIN / FILTER_MEDIAN)
    over the offsets where the dense (2r+1)^ndim mask is nonzero. Values are
    ordered numerically with -0 below +0; a window holding a NaN gives NaN;
    the median of m values is the element of rank (m-1)//2. Returns a padded
    array, halo zero."""
    nd, n = _dims(a, r)
    mask = np.ascontiguousarray(mask, dtype=np.float64)
    assert mask.shape == (2 * r + 1,) * nd
    out = np.zeros_like(a)
    if lib().oracle_filter(_ptr(a), _ptr(out), nd, n, r, _ptr(mask), int(op)) != 0:
        raise ValueError("unknown filter op")
    return out


def filter_at(a, r, mask, op, pts):
    """The window filter at interior points pts (rows of (x, y, z))."""
    nd, n = _dims(a, r)
    mask = np.ascontiguousarray(mask, dtype=np.float64)
    assert mask.shape == (2 * r + 1,) * nd
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    nn = [n[0], n[1], n[2]]
    if len(pts) and (pts.min() < 0 or any(pts[:, a].max() >= nn[a] for a in range(3))):
        raise ValueError("point outside the interior")
    out = np.zeros(len(pts))
    if lib().oracle_filter_at(_ptr(a), nd, n, r, _ptr(mask), int(op), pts.ctypes.data_as(_lp),
                              len(pts), _ptr(out)) != 0:
        raise ValueError("unknown filter op")
    return out


def xcorr_at(a, r, g, pts):
    """Cross-correlation at interior points pts (array of (x, y, z) rows)."""
    nd, n = _dims(a, r)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (2 * r + 1,) * nd
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    nn = [n[0], n[1], n[2]]
    if len(pts) and (pts.min() < 0 or any(pts[:, a].max() >= nn[a] for a in range(3))):
        raise ValueError("point outside the interior")
    out = np.zeros(len(pts))
    lib().oracle_xcorr_at(_ptr(a), nd, n, r, _ptr(g), pts.ctypes.data_as(_lp), len(pts),
                          _ptr(out))
    return out


# --------------------------------------------------------------------------
# sixth-order derivatives, right-hand sides, RK3
# --------------------------------------------------------------------------

def fd_weights():
    c1 = np.zeros(7)
    c2 = np.zeros(7)
    lib().oracle_fd_weights(_ptr(c1), _ptr(c2))
    return c1, c2


def rk3_coeffs():
    a = np.zeros(3)
    b = np.zeros(3)
    lib().oracle_rk3_coeffs(_ptr(a), _ptr(b))
    return a, b


def deriv(f, ds, op):
    """Apply derivative operator ``op`` to radius-3 padded field f."""
    nd, n = _dims(f, 3)
    out = np.zeros_like(f)
    if lib().oracle_deriv(_ptr(f), _ptr(out), nd, n, _d3(ds), op) != 0:
        raise ValueError("operator not defined in %d dimensions" % nd)
    return out


def _model_prm(model, nu, eta, cs2, c, mhd=None):
    if model == MODEL_MHD8:
        return (ctypes.c_double * 4)(nu, eta, cs2, 0.0)
    if model == MODEL_MHD_FULL:
        m = dict(MHD_DEFAULTS, **(mhd or {}))
        return (ctypes.c_double * 11)(nu, eta, cs2, m["zeta"], m["mu0"], m["gamma"], m["cp"],
                                      m["lnrho0"], m["K"], m["heat"], m["cool"])
    c = list(c) + [0.0] * (3 - len(c))
    return (ctypes.c_double * 4)(nu, *c)


def _nf(model):
    return 1 if model == MODEL_ADVDIFF else 8


def _code(model, mixed):
    """Model code for the C oracle: the MHD models take the bank's mixed
    derivatives from the tensor product (default) or the diagonals."""
    if mixed == MIXED_TENSOR:
        return model
    if mixed == MIXED_DIAG and model != MODEL_ADVDIFF:
        return model | 0x100
    raise ValueError("mixed must be 'tensor' or 'diag' (MHD models only)")


def rhs(model, fields, ds, nu=1e-3, eta=1e-3, cs2=1.0, c=(0.0, 0.0, 0.0), mhd=None,
        mixed=MIXED_TENSOR):
    """Right-hand side R of the model over the interior; returns padded arrays
    (halo zero), one per field. For MODEL_MHD_FULL, cs2 is cs0^2 and mhd
    overrides MHD_DEFAULTS. mixed selects the bank's mixed derivatives."""
    nd, n = _dims(fields[0], 3)
    if len(fields) != _nf(model):
        raise ValueError("wrong number of fields for the model")
    R = [np.zeros_like(fields[0]) for _ in fields]
    rc = lib().oracle_rhs(_code(model, mixed), _ptrs(fields), _ptrs(R), nd, n, _d3(ds),
                          _model_prm(model, nu, eta, cs2, c, mhd))
    if rc != 0:
        raise ValueError("bad model/dimension")
    return R


def rk3_substep(model, stage, fin, w, ds, dt, nu=1e-3, eta=1e-3, cs2=1.0,
                c=(0.0, 0.0, 0.0), mhd=None, mixed=MIXED_TENSOR):
    """One Williamson substep: updates the arrays in w in place and returns
    new padded f arrays with a periodic halo."""
    nd, n = _dims(fin[0], 3)
    if len(fin) != len(w) or len(fin) != _nf(model):
        raise ValueError("wrong number of fields for the model")
    if any(a.shape != fin[0].shape for a in w):
        raise ValueError("w must match the fields' padded shape")
    fout = [np.zeros_like(a) for a in fin]
    rc = lib().oracle_rk3_substep(_code(model, mixed), stage, _ptrs(fin), _ptrs(w),
                                  _ptrs(fout), nd, n,
                                  _d3(ds), _model_prm(model, nu, eta, cs2, c, mhd), dt)
    if rc != 0:
        raise ValueError("bad model/dimension/stage")
    return fout


def rk3_steps(model, f, ds, dt, steps, **kw):
    """``steps`` full RK3 steps from padded f (halo refreshed first); returns
    the final padded fields. The inputs are not modified."""
    cur = [fill_periodic(a.copy(), 3) for a in f]
    w = [np.zeros_like(a) for a in f]
    for _ in range(steps):
        for stage in range(3):
            cur = rk3_substep(model, stage, cur, w, ds, dt, **kw)
    return cur


def rk3_substep_at(model, stage, fin, w_in, ds, dt, pts, nu=1e-3, eta=1e-3, cs2=1.0,
                   c=(0.0, 0.0, 0.0), mhd=None, mixed=MIXED_TENSOR):
    """Substep at listed interior points. w_in: (nf, count) old w (ignored at
    stage 0). Returns (w_out, f_out), each (nf, count)."""
    nd, n = _dims(fin[0], 3)
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    nf = len(fin)
    if nf != _nf(model):
        raise ValueError("wrong number of fields for the model")
    nn = [n[0], n[1], n[2]]
    if len(pts) and (pts.min() < 0 or any(pts[:, a].max() >= nn[a] for a in range(3))):
        raise ValueError("point outside the interior")
    cnt = len(pts)
    w_in = np.ascontiguousarray(np.zeros((nf, cnt)) if w_in is None else w_in,
                                dtype=np.float64)
    w_out = np.zeros((nf, cnt))
    f_out = np.zeros((nf, cnt))
    rc = lib().oracle_rk3_substep_at(_code(model, mixed), stage, _ptrs(fin), _ptr(w_in), nd, n,
                                     _d3(ds),
                                     _model_prm(model, nu, eta, cs2, c, mhd), dt,
                                     pts.ctypes.data_as(_lp), cnt, _ptr(w_out), _ptr(f_out))
    if rc != 0:
        raise ValueError("bad model/dimension/stage")
    return w_out, f_out


def reduce(f, r):
    """(sum, sum of squares, max |f|) over the interior, sequential FP64."""
    nd, n = _dims(f, r)
    out = np.zeros(3)
    lib().oracle_reduce(_ptr(f), nd, n, r, _ptr(out))
    return out


def energy(fields, ds):
    """(1/2 sum |u|^2, 1/2 sum |curl A|^2) over the interior of the 8 padded
    MHD fields (Table A1 order, periodic halos), sixth-order first
    derivatives, sequential FP64 sums over grid points."""
    nd, n = _dims(fields[0], 3)
    if nd != 3 or len(fields) != 8:
        raise ValueError("needs the 8 padded 3-D MHD fields")
    out = np.zeros(2)
    lib().oracle_energy(_ptrs(fields), n, _d3(ds), _ptr(out))
    return out
