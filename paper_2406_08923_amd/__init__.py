"""Python binding of libstencil.so (MI355X / gfx950 stencil library).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/stencil.h. PyTorch supplies the
device memory (tensors) and streams; tensors are passed as raw pointers.

The library is loaded lazily on first use, after ``import torch`` so that the
process has a single HIP runtime. There is no fallback: if libstencil.so is
missing or fails to load, the call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil.so")

# storage types, boundary modes, variants (include/stencil.h)
F64, F32, BF16 = 0, 1, 2
PERIODIC, USER_HALO = 0, 1
VARIANT_AUTO, GENERIC, STAR3D, LINE1D, BOX3D = -1, 0, 1, 2, 3
# stencil function: cross-correlation, or a window filter (max filter of
# Sec. 2.3, its min twin, median filter of Sec. 1)
OP_XCORR, OP_MAX, OP_MIN, OP_MEDIAN = 0, 1, 2, 3
MEDIAN_MAX = 27
FLAG_AUTOTUNE = 1
APPLY_HALO_VALID = 1

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EUNSUPPORTED", -4: "EDEVICE",
           -5: "EAGAIN", -6: "ESTATE", -7: "ETIMEOUT"}


class StencilError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("dims", ctypes.c_int * 3), ("radius", ctypes.c_int),
                ("coeffs", ctypes.POINTER(ctypes.c_double)), ("dtype", ctypes.c_int),
                ("bc", ctypes.c_int), ("flags", ctypes.c_uint), ("variant", ctypes.c_int),
                ("tile", ctypes.c_int * 4), ("row_pitch", ctypes.c_int),
                ("x_offset", ctypes.c_int), ("op", ctypes.c_int)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded libstencil.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstencil.so is not built: run __graft_entry__.build() "
                               "or python paper_2406_08923_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    c_int, c_size = ctypes.c_int, ctypes.c_size_t
    L.stencil_last_error.restype = ctypes.c_char_p
    L.stencil_version.restype = c_int
    L.stencil_padded_elems.argtypes = [c_int, ctypes.POINTER(c_int), c_int]
    L.stencil_padded_elems.restype = c_size
    L.stencil_plan_padded_elems.argtypes = [_vp]
    L.stencil_plan_padded_elems.restype = c_size
    L.stencil_plan_halo.argtypes = [_vp, _vp, _vp]
    L.stencil_plan.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_vp)]
    L.stencil_plan_destroy.argtypes = [_vp]
    L.stencil_plan_variant.argtypes = [_vp]
    L.stencil_plan_tile.argtypes = [_vp, ctypes.POINTER(c_int)]
    L.stencil_apply.argtypes = [_vp, _vp, _vp, c_int, _vp]
    L.stencil_apply_ex.argtypes = [_vp, _vp, _vp, c_int, ctypes.c_uint, _vp]
    L.stencil_halo_periodic.argtypes = [c_int, ctypes.POINTER(c_int), c_int, c_int, _vp, _vp]
    L.stencil_copy.argtypes = [_vp, _vp, c_size, _vp]
    L.stencil_fd_weights.argtypes = [c_int, c_int, ctypes.POINTER(ctypes.c_double)]
    _declare_rk(L)
    _declare_server(L)


def check(rc):
    if rc != 0:
        msg = lib().stencil_last_error()
        raise StencilError(rc, msg.decode() if msg else "")
    return rc


def stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def ptr(t):
    return _vp(t.data_ptr())


def torch_dtype(dtype):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[dtype]


def _dims3(dims):
    d = list(dims) + [1] * (3 - len(dims))
    return (ctypes.c_int * 3)(*d)


def padded_elems(dims, radius):
    return int(lib().stencil_padded_elems(len(dims), _dims3(dims), radius))


def padded_shape(dims, radius):
    """Tensor shape [z, y, x] (slowest first) of a padded field."""
    return tuple(int(dims[k]) + 2 * radius for k in reversed(range(len(dims))))


def fd_weights(order, radius):
    out = (ctypes.c_double * (2 * radius + 1))()
    check(lib().stencil_fd_weights(order, radius, out))
    return np.array(out[:])


def halo_periodic(buf, dims, radius, dtype, stream=None):
    check(lib().stencil_halo_periodic(len(dims), _dims3(dims), radius, dtype, ptr(buf),
                                      stream_ptr(stream)))


def copy(src, dst, nbytes=None, stream=None):
    n = src.numel() * src.element_size() if nbytes is None else nbytes
    check(lib().stencil_copy(ptr(src), ptr(dst), n, stream_ptr(stream)))


class LinearPlan:
    """Plan of a linear stencil (Eq. 3 / Eq. 6-7): ``coeffs`` is the dense
    (2r+1)^ndim tensor in NumPy order [s_z, s_y, s_x] (x fastest). With op
    OP_MAX / OP_MIN / OP_MEDIAN the plan is a window filter over the offsets
    where coeffs is nonzero."""

    def __init__(self, dims, radius, coeffs, dtype=F64, bc=PERIODIC, autotune=False,
                 variant=VARIANT_AUTO, tile=None, row_pitch=0, x_offset=0, op=OP_XCORR):
        self.dims = tuple(int(v) for v in dims)
        self.ndim = len(self.dims)
        self.radius = int(radius)
        self.dtype = dtype
        self.x_offset = int(x_offset) or self.radius
        self.row_pitch = int(row_pitch) or (self.x_offset + self.dims[0] + self.radius)
        c = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(-1)
        if c.size != (2 * radius + 1) ** self.ndim:
            raise ValueError("coeffs must hold (2r+1)^ndim values")
        self._coeffs = c
        d = _Desc()
        d.ndim = self.ndim
        d.dims = _dims3(self.dims)
        d.radius = self.radius
        d.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.dtype = dtype
        d.bc = bc
        d.flags = FLAG_AUTOTUNE if autotune else 0
        d.variant = variant
        d.tile = (ctypes.c_int * 4)(*(list(tile or []) + [0] * 4)[:4])
        d.row_pitch = int(row_pitch)
        d.x_offset = int(x_offset)
        d.op = int(op)
        self.op = int(op)
        h = _vp()
        check(lib().stencil_plan(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @property
    def variant(self):
        v = lib().stencil_plan_variant(self._h)
        return check(v) if v < 0 else v

    @property
    def tile(self):
        t = (ctypes.c_int * 4)()
        check(lib().stencil_plan_tile(self._h, t))
        return tuple(t)

    def reduce(self, fields, dtype=None, stream=None):
        """(sum, sum of squares, max |f|) per buffer, FP64, deterministic."""
        dtype = self.dtype if dtype is None else dtype
        ptrs = (_vp * len(fields))(*[t.data_ptr() for t in fields])
        out = (ctypes.c_double * (3 * len(fields)))()
        check(lib().stencil_reduce(self._h, ptrs, len(fields), dtype, out, stream_ptr(stream)))
        return np.array(out[:]).reshape(len(fields), 3)

    @property
    def iterations_per_launch(self):
        """Chained iterations one kernel launch performs (2 for a periodic
        star planned with temporal blocking, else 1)."""
        if self.variant == STAR3D:
            return 2 if (self.tile[3] >> 12) & 15 == 2 else 1
        if self.variant == LINE1D:
            return max(1, self.tile[1])
        return 1

    def launches(self, iters):
        """(launches of the multi-iteration kernel, one-iteration launches)
        that apply(a, b, iters) issues for a two-iteration star plan: the
        launch count has the parity of iters, so the result lands where the
        one-iteration-per-launch contract puts it."""
        if self.iterations_per_launch != 2 or self.variant != STAR3D:
            return 0, iters
        nl = (iters + 1) // 2
        if nl % 2 != iters % 2:
            nl += 1
        return iters - nl, 2 * nl - iters

    @property
    def storage_shape(self):
        """Tensor shape [z, y, x] of one field in the plan's layout (rows of
        row_pitch elements)."""
        return padded_shape(self.dims, self.radius)[:-1] + (self.row_pitch,)

    def padded(self, t):
        """View of the padded field (Eq. 2 extents) inside a storage tensor:
        columns [x_offset - r, x_offset + nx + r) of every row."""
        lo = self.x_offset - self.radius
        return t[..., lo:lo + self.dims[0] + 2 * self.radius]

    def empty(self, fill=None):
        """A device tensor of the plan's storage shape and dtype."""
        import torch
        t = torch.empty(self.storage_shape, dtype=torch_dtype(self.dtype), device="cuda")
        if fill is not None:
            t.fill_(fill)
        return t

    def halo(self, t, stream=None):
        """Periodic halo refresh of one field in the plan's layout."""
        self._check_buf(t)
        check(lib().stencil_plan_halo(self._h, ptr(t), stream_ptr(stream)))

    def _check_buf(self, t):
        n = int(lib().stencil_plan_padded_elems(self._h))
        if t.numel() != n or not t.is_contiguous() or t.dtype != torch_dtype(self.dtype):
            raise ValueError("buffer must be a contiguous tensor of the plan's storage shape "
                             "and dtype")

    def apply(self, a, b, iters=1, stream=None, halo_valid=False):
        """Chained application; the result is in b for odd iters, else in a.
        halo_valid: a's periodic halo is already valid (no refresh launch)."""
        n = int(lib().stencil_plan_padded_elems(self._h))
        for t in (a, b):
            if t.numel() != n or not t.is_contiguous() or t.dtype != torch_dtype(self.dtype):
                raise ValueError("buffer must be a contiguous padded tensor of the plan dtype")
        check(lib().stencil_apply_ex(self._h, ptr(a), ptr(b), int(iters),
                                     APPLY_HALO_VALID if halo_valid else 0, stream_ptr(stream)))
        return b if iters % 2 else a

    def close(self):
        if getattr(self, "_h", None):
            lib().stencil_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# fused nonlinear substep (derivative bank + phi + low-storage RK3)
# ---------------------------------------------------------------------------

MODEL_MHD8, MODEL_ADVDIFF, MODEL_MHD_FULL = 0, 1, 2
# mixed derivatives of the MHD banks: tensor product (36 taps) or diagonals (12)
MIXED_TENSOR, MIXED_DIAGONAL = 0, 1
# constants of MODEL_MHD_FULL beyond nu, eta and cs2 (= cs0^2); a plan's mhd
# dict overrides any of them
MHD_FULL_DEFAULTS = dict(zeta=0.0, mu0=1.0, gamma=5.0 / 3.0, cp=1.0, lnrho0=0.0, K=0.0,
                         heat=0.0, cool=0.0)
RK_AUTO, RK_CACHED, RK_LDS = 0, 1, 2
PREC_F64, PREC_F32_MASTER64, PREC_BF16_MASTER64, PREC_F32_ONLY, PREC_BF16_ONLY = range(5)
_PREC_STORE = {PREC_F64: F64, PREC_F32_MASTER64: F32, PREC_BF16_MASTER64: BF16,
               PREC_F32_ONLY: F32, PREC_BF16_ONLY: BF16}


class _RkDesc(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("ndim", ctypes.c_int), ("dims", ctypes.c_int * 3),
                ("precision", ctypes.c_int), ("ds", ctypes.c_double * 3),
                ("nu", ctypes.c_double), ("eta", ctypes.c_double), ("cs2", ctypes.c_double),
                ("adv", ctypes.c_double * 3), ("block", ctypes.c_int * 3),
                ("variant", ctypes.c_int), ("row_pitch", ctypes.c_int),
                ("x_offset", ctypes.c_int)] + [
                    (k, ctypes.c_double) for k in ("zeta", "mu0", "gamma", "cp", "lnrho0", "K",
                                                   "heat", "cool")] + [
                    ("mixed", ctypes.c_int), ("flags", ctypes.c_uint), ("occupancy", ctypes.c_int)]


RK_FLAG_AUTOTUNE = 1


class _Fields(ctypes.Structure):
    _fields_ = [("f_in", _vp * 8), ("f_out", _vp * 8), ("w", _vp * 8), ("w2", _vp * 8),
                ("f64", _vp * 8)]


def _declare_rk(L):
    c_int = ctypes.c_int
    L.stencil_plan_rk.argtypes = [ctypes.POINTER(_RkDesc), ctypes.POINTER(_vp)]
    L.stencil_plan_nfields.argtypes = [_vp]
    L.stencil_plan_rk_schedule.argtypes = [_vp, ctypes.POINTER(c_int)]
    L.stencil_step.argtypes = [_vp, ctypes.POINTER(_Fields), c_int, ctypes.c_double, _vp]
    L.stencil_rk_run.argtypes = [_vp, ctypes.POINTER(_Fields), c_int, ctypes.c_double, _vp]
    L.stencil_reduce.argtypes = [_vp, ctypes.POINTER(_vp), c_int, c_int,
                                 ctypes.POINTER(ctypes.c_double), _vp]
    L.stencil_reduce_noalloc.argtypes = [_vp, ctypes.POINTER(_vp), c_int, c_int,
                                         ctypes.POINTER(ctypes.c_double), _vp]
    L.stencil_energy.argtypes = [_vp, ctypes.POINTER(_vp), c_int,
                                 ctypes.POINTER(ctypes.c_double), _vp]


def _fields_struct(f_in, f_out, w, w2=None, f64=None):
    fs = _Fields()
    for name, lst in (("f_in", f_in), ("f_out", f_out), ("w", w), ("w2", w2), ("f64", f64)):
        if lst is None:
            continue
        arr = getattr(fs, name)
        for k, t in enumerate(lst):
            arr[k] = t.data_ptr() if t is not None else None
    return fs


class RkPlan:
    """Plan of the fused substep of a model (MODEL_MHD8, MODEL_MHD_FULL: 8
    fields, 3-D; MODEL_ADVDIFF: 1 field, 2-D or 3-D), radius-3 periodic
    padding. For MODEL_MHD_FULL, cs2 is cs0^2 and mhd overrides
    MHD_FULL_DEFAULTS. mixed (MHD models): MIXED_TENSOR or MIXED_DIAGONAL
    mixed derivatives in the bank."""

    def __init__(self, model, dims, precision=PREC_F64, ds=None, nu=1e-3, eta=1e-3, cs2=1.0,
                 adv=(0.0, 0.0, 0.0), block=None, variant=0, row_pitch=0, x_offset=0,
                 mhd=None, mixed=MIXED_TENSOR, autotune=False, occupancy=0):
        import math
        self.model = model
        self.dims = tuple(int(v) for v in dims)
        self.ndim = len(self.dims)
        self.precision = precision
        self.dtype = _PREC_STORE[precision]
        self.master = precision in (PREC_F32_MASTER64, PREC_BF16_MASTER64)
        if ds is None:
            ds = [2 * math.pi / v for v in self.dims]
        d = _RkDesc()
        d.model = model
        d.ndim = self.ndim
        d.dims = _dims3(self.dims)
        d.precision = precision
        d.ds = (ctypes.c_double * 3)(*(list(ds) + [1.0] * (3 - len(ds))))
        d.nu, d.eta, d.cs2 = nu, eta, cs2
        d.adv = (ctypes.c_double * 3)(*(list(adv) + [0.0] * (3 - len(adv))))
        d.block = (ctypes.c_int * 3)(*(list(block or []) + [0, 0, 0])[:3])
        d.variant = int(variant)
        self.variant = int(variant)
        d.row_pitch = int(row_pitch)
        d.x_offset = int(x_offset)
        unknown = set(mhd or {}) - set(MHD_FULL_DEFAULTS)
        if unknown:
            raise ValueError("unknown MHD constants %s" % sorted(unknown))
        for k, v in dict(MHD_FULL_DEFAULTS, **(mhd or {})).items():
            setattr(d, k, float(v))
        d.mixed = int(mixed)
        self.mixed = int(mixed)
        d.flags = RK_FLAG_AUTOTUNE if autotune else 0
        d.occupancy = int(occupancy)
        self.x_offset = int(x_offset) or 3
        self.row_pitch = int(row_pitch) or (self.x_offset + self.dims[0] + 3)
        L = lib()
        h = _vp()
        check(L.stencil_plan_rk(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.nfields = L.stencil_plan_nfields(h)

    @property
    def schedule(self):
        """(variant, bx, by, bz, occupancy) the plan launches (after any
        search)."""
        out = (ctypes.c_int * 5)()
        check(lib().stencil_plan_rk_schedule(self._h, out))
        return tuple(out)

    @property
    def reg_dtype(self):
        import torch
        return torch.float64 if self.precision == PREC_F64 else torch.float32

    def alloc(self):
        """Device buffers of one integration: f_a, f_b (storage), w, w2
        (registers) and f64 (master), as lists of padded tensors."""
        import torch
        shp = self.storage_shape
        sd = torch_dtype(self.dtype)
        mk = lambda dt: [torch.zeros(shp, dtype=dt, device="cuda") for _ in range(self.nfields)]
        bufs = {"f_a": mk(sd), "f_b": mk(sd), "w": mk(self.reg_dtype)}
        bufs["w2"] = mk(self.reg_dtype) if self.master else None
        bufs["f64"] = mk(torch.float64) if self.master else None
        return bufs

    @property
    def storage_shape(self):
        """Tensor shape [z, y, x] of one buffer in the plan's layout."""
        return padded_shape(self.dims, 3)[:-1] + (self.row_pitch,)

    def padded(self, t):
        """View of the padded field (extents n + 6) inside a storage tensor."""
        lo = self.x_offset - 3
        return t[..., lo:lo + self.dims[0] + 6]

    def interior(self, t):
        """View of the interior points inside a storage tensor."""
        return self.padded(t)[(slice(3, -3),) * self.ndim]

    def step(self, f_in, f_out, w, substep, dt, w2=None, f64=None, stream=None):
        fs = _fields_struct(f_in, f_out, w, w2, f64)
        check(lib().stencil_step(self._h, ctypes.byref(fs), int(substep), float(dt),
                                 stream_ptr(stream)))

    def run(self, f_a, f_b, w, nsteps, dt, w2=None, f64=None, stream=None):
        """nsteps full steps; returns the list holding the result."""
        fs = _fields_struct(f_a, f_b, w, w2, f64)
        check(lib().stencil_rk_run(self._h, ctypes.byref(fs), int(nsteps), float(dt),
                                   stream_ptr(stream)))
        return f_b if nsteps % 2 else f_a

    def reduce(self, fields, dtype=None, stream=None):
        """(sum, sum of squares, max |f|) per field, FP64, deterministic."""
        dtype = self.dtype if dtype is None else dtype
        ptrs = (_vp * len(fields))(*[t.data_ptr() for t in fields])
        out = (ctypes.c_double * (3 * len(fields)))()
        check(lib().stencil_reduce(self._h, ptrs, len(fields), dtype, out, stream_ptr(stream)))
        return np.array(out[:]).reshape(len(fields), 3)

    def reduce_noalloc(self, fields, dtype=None, stream=None):
        """reduce() without device allocation (the library's fixed scratch
        array; calls overlapping on one GPU race)."""
        dtype = self.dtype if dtype is None else dtype
        ptrs = (_vp * len(fields))(*[t.data_ptr() for t in fields])
        out = (ctypes.c_double * (3 * len(fields)))()
        check(lib().stencil_reduce_noalloc(self._h, ptrs, len(fields), dtype, out,
                                           stream_ptr(stream)))
        return np.array(out[:]).reshape(len(fields), 3)

    def energy(self, fields, dtype=None, stream=None):
        """(1/2 sum |u|^2, 1/2 sum |curl A|^2) of the 8 MHD fields (padded
        buffers with valid halos), FP64, deterministic."""
        dtype = self.dtype if dtype is None else dtype
        if len(fields) != 8:
            raise ValueError("energy needs the 8 MHD fields")
        ptrs = (_vp * 8)(*[t.data_ptr() for t in fields])
        out = (ctypes.c_double * 2)()
        check(lib().stencil_energy(self._h, ptrs, dtype, out, stream_ptr(stream)))
        return np.array(out[:])

    def close(self):
        if getattr(self, "_h", None):
            lib().stencil_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batched jobs and the serving loop
# ---------------------------------------------------------------------------

JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = range(5)
# order in which a server tick takes resident jobs (stencil_server_desc.policy)
SERVE_OLDEST, SERVE_SHORTEST = 0, 1


class _Job(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("dims", ctypes.c_int * 3), ("steps", ctypes.c_int),
                ("precision", ctypes.c_int), ("nu", ctypes.c_double),
                ("adv", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("init", ctypes.POINTER(ctypes.c_double)),
                ("result", ctypes.POINTER(ctypes.c_double))]


class _JobStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("error", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_first_tick", ctypes.c_double),
                ("t_done", ctypes.c_double), ("steps_done", ctypes.c_longlong)]


class _ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("tick_steps", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("blocks", ctypes.c_int), ("queue_cap", ctypes.c_int),
                ("min_points", ctypes.c_longlong), ("policy", ctypes.c_int),
                ("tune", ctypes.c_int)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_longlong), ("launches", ctypes.c_longlong),
                ("admitted", ctypes.c_longlong), ("completed", ctypes.c_longlong),
                ("failed", ctypes.c_longlong), ("cancelled", ctypes.c_longlong),
                ("point_steps", ctypes.c_longlong), ("bytes_in_use", ctypes.c_size_t),
                ("bytes_budget", ctypes.c_size_t), ("resident", ctypes.c_int),
                ("queued", ctypes.c_int), ("busy_s", ctypes.c_double),
                ("tuned_classes", ctypes.c_int)]


def _declare_server(L):
    u64 = ctypes.c_uint64
    L.stencil_server_create.argtypes = [ctypes.POINTER(_ServerDesc), ctypes.POINTER(_vp)]
    L.stencil_server_destroy.argtypes = [_vp]
    L.stencil_submit.argtypes = [_vp, ctypes.POINTER(_Job), ctypes.POINTER(u64)]
    L.stencil_poll.argtypes = [_vp, u64, ctypes.POINTER(_JobStatus)]
    L.stencil_wait.argtypes = [_vp, u64, ctypes.POINTER(_JobStatus), ctypes.c_int]
    L.stencil_cancel.argtypes = [_vp, u64]
    L.stencil_server_stats_get.argtypes = [_vp, ctypes.POINTER(_ServerStats)]
    L.stencil_server_clock.argtypes = [_vp]
    L.stencil_server_clock.restype = ctypes.c_double


def _status_dict(s):
    return {"state": s.state, "error": s.error, "t_submit": s.t_submit, "t_admit": s.t_admit,
            "t_first_tick": s.t_first_tick, "t_done": s.t_done, "steps_done": s.steps_done}


class Server:
    """Continuous-batching server of scalar advection-diffusion jobs. Initial
    states and result arrays are NumPy float64 interiors ([z,] y, x order);
    they are kept referenced until the job ends."""

    def __init__(self, hbm_budget=0, max_slots=256, tick_steps=10, use_graph=True, blocks=0,
                 queue_cap=0, min_points=0, policy=SERVE_OLDEST, tune=False):
        L = lib()
        d = _ServerDesc(hbm_budget, max_slots, tick_steps, 1 if use_graph else 0, blocks,
                        queue_cap, min_points, policy, 1 if tune else 0)
        h = _vp()
        check(L.stencil_server_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, init, steps, precision=PREC_F64, nu=1e-3, adv=(0.0, 0.0, 0.0), dt=0.0,
               result=None):
        init = np.ascontiguousarray(init, dtype=np.float64)
        nd = init.ndim
        if result is None:
            result = np.empty_like(init)
        j = _Job()
        j.ndim = nd
        j.dims = _dims3([init.shape[nd - 1 - k] for k in range(nd)])
        j.steps = int(steps)
        j.precision = precision
        j.nu = nu
        j.adv = (ctypes.c_double * 3)(*(list(adv) + [0.0] * (3 - len(adv))))
        j.dt = dt
        j.init = init.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        j.result = result.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        t = ctypes.c_uint64()
        check(lib().stencil_submit(self._h, ctypes.byref(j), ctypes.byref(t)))
        self._keep[t.value] = (init, result)
        return t.value

    def result(self, ticket):
        return self._keep[ticket][1]

    def poll(self, ticket):
        s = _JobStatus()
        check(lib().stencil_poll(self._h, ticket, ctypes.byref(s)))
        return _status_dict(s)

    def wait(self, ticket, timeout_ms=-1):
        s = _JobStatus()
        rc = lib().stencil_wait(self._h, ticket, ctypes.byref(s), int(timeout_ms))
        if rc not in (0, -7):
            check(rc)
        d = _status_dict(s)
        d["timed_out"] = rc == -7
        return d

    def cancel(self, ticket):
        check(lib().stencil_cancel(self._h, ticket))

    def stats(self):
        s = _ServerStats()
        check(lib().stencil_server_stats_get(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def clock(self):
        return lib().stencil_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().stencil_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
