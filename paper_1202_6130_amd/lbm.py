"""Python binding of the lbm C ABI (include/lbm.h).

Argument marshalling only: every step of the update runs in the HIP library
liblbmwet.so.  PyTorch supplies the device workspace (a uint8 tensor) and the
current HIP stream.  Importing this module does not load the library; the
first call does, and raises if it is missing or was built for nothing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblbmwet.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ENOFIT, LBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
STORE_F32, STORE_F16DEV, STORE_F64, STORE_F32X = 0, 1, 2, 3
WALL_NONE, WALL_FLAT_SLAB, WALL_FIELDS, WALL_MASK = 0, 1, 2, 3
D2Q9, D2Q21 = 9, 21
PSI_EXP, PSI_EOS = 0, 1
COLL_BGK, COLL_PROJECTED = 0, 1

_NAMES = {LBM_EINVAL: "EINVAL", LBM_ENOMEM: "ENOMEM", LBM_EDEVICE: "EDEVICE", LBM_EUNSTABLE: "EUNSTABLE",
          LBM_ENOFIT: "ENOFIT", LBM_ESTATE: "ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm {_NAMES.get(code, code)}: {msg}")
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("wall_kind", ctypes.c_int32),
                ("tau", ctypes.c_double), ("G", ctypes.c_double),
                ("G_R", ctypes.c_double), ("G_A", ctypes.c_double), ("eps", ctypes.c_double),
                ("U_wall", ctypes.c_double * 2), ("F_ext", ctypes.c_double * 2),
                ("wall_width", ctypes.c_double), ("core_range", ctypes.c_double),
                ("tail_range", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("slab_rows", ctypes.c_int32), ("diag_interval", ctypes.c_int32),
                ("seg_rows", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("psi_kind", ctypes.c_int32), ("eos", ctypes.c_double * 5),
                ("collision", ctypes.c_int32), ("filter_core", ctypes.c_int32), ("filter_wall", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


def lib():
    """Load liblbmwet.so (in-tree build).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_1202_6130_amd.build)")
    # PyTorch bundles its own HIP runtime with the same soname as the system
    # one.  Load torch first so the library binds to that runtime: one
    # process must not hold two HIP runtimes (workspace and streams come from
    # torch).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lbm_params)
    i64 = ctypes.c_int64
    sig = {
        "lbm_params_default": ([P], ctypes.c_int),
        "lbm_last_error": ([_vp], ctypes.c_char_p),
        "lbm_workspace_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_device_copy": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
        "lbm_create": ([P, _dp, _dp, _dp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
        "lbm_step": ([_vp, i64, _dp], ctypes.c_int),
        "lbm_diagnostics": ([_vp, _dp], ctypes.c_int),
        "lbm_diagnostics_noalloc": ([_vp, _dp], ctypes.c_int),
        "lbm_moments": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int),
        "lbm_contact_angle": ([_vp, ctypes.c_double, ctypes.c_double, _dp], ctypes.c_int),
        "lbm_slip_length": ([_vp, _dp], ctypes.c_int),
        "lbm_dynamic_angles": ([_vp, ctypes.c_double, ctypes.c_double, _dp], ctypes.c_int),
        "lbm_get_state": ([_vp, _dp], ctypes.c_int),
        "lbm_set_state": ([_vp, _dp, i64], ctypes.c_int),
        "lbm_step_index": ([_vp], i64),
        "lbm_destroy": ([_vp], ctypes.c_int),
        "lbm_batch_workspace_bytes": ([P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_batch_create": ([P, ctypes.c_int32, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                              ctypes.c_int32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
        "lbm_batch_step": ([_vp, i64, ctypes.c_int32], ctypes.c_int),
        "lbm_batch_diagnostics": ([_vp, _dp], ctypes.c_int),
        "lbm_batch_lattice": ([_vp, ctypes.c_int32], _vp),
        "lbm_batch_destroy": ([_vp], ctypes.c_int),
        "lbm_batch_attach_bytes": ([ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
        "lbm_batch_attach": ([ctypes.POINTER(_vp), ctypes.c_int32, _vp, ctypes.c_size_t, _vp,
                              ctypes.POINTER(_vp)], ctypes.c_int),
        "lbm_tile_shapes": ([_ip, _ip, _ip, ctypes.c_int32], ctypes.c_int32),
        "lbm_set_tile_shape": ([_vp, ctypes.c_int32], ctypes.c_int),
        "lbm_get_tile_shape": ([_vp], ctypes.c_int32),
        "lbm_two_step_variants": ([_ip, _ip, _ip, ctypes.c_int32], ctypes.c_int32),
        "lbm_set_two_step": ([_vp, ctypes.c_int32], ctypes.c_int),
        "lbm_get_two_step": ([_vp], ctypes.c_int32),
        "lbm_tune_two_step": ([_vp, ctypes.c_int32, _ip, _dp], ctypes.c_int),
        "lbm_tune": ([_vp, ctypes.c_int32, _ip, _dp], ctypes.c_int),
        "lbm_batch_set_tile_shapes": ([_vp, _ip], ctypes.c_int),
        "lbm_batch_get_tile_shapes": ([_vp, _ip], ctypes.c_int),
        "lbm_batch_tune": ([_vp, ctypes.c_int32, _ip, _dp], ctypes.c_int),
        "lbm_batch_set_two_step": ([_vp, ctypes.c_int32], ctypes.c_int),
        "lbm_batch_get_two_step": ([_vp], ctypes.c_int32),
        "lbm_batch_tune_two_step": ([_vp, ctypes.c_int32, _ip, _dp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return _lib


def _check(code):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_last_error(None).decode())
    return code


def lbm_last_error(ctx=None):
    """Message of the last failed call on ctx, or of the calling thread."""
    return lib().lbm_last_error(ctx).decode()


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "float64 C-contiguous array required"
    return a.ctypes.data_as(_dp)


def _iptr(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"], "int32 C-contiguous array required"
    return a.ctypes.data_as(_ip)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _u0(ux0, uy0):
    """Initial velocity as the [2, ny, nx] array of lbm_create (None at rest)."""
    if ux0 is None and uy0 is None:
        return None
    if ux0 is None or uy0 is None:
        raise ValueError("give both ux0 and uy0, or neither")
    return np.ascontiguousarray(np.stack([np.asarray(ux0, dtype=np.float64), np.asarray(uy0, dtype=np.float64)]))


# ------------------------------------------------------------ C names
def lbm_params_default(**kw):
    p = lbm_params()
    _check(lib().lbm_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k in ("U_wall", "F_ext", "eos"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def nq(p):
    """Populations per node of the parameters' velocity set."""
    return 21 if p.lattice == D2Q21 else 9


def lbm_device_copy(src_ptr, dst_ptr, nbytes, stream_ptr):
    """Plain 16-byte non-temporal device copy (the bandwidth reference);
    device pointers and the stream as integers."""
    _check(lib().lbm_device_copy(_vp(src_ptr), _vp(dst_ptr), ctypes.c_size_t(nbytes), _vp(stream_ptr)))


def lbm_workspace_bytes(p):
    n = ctypes.c_size_t()
    _check(lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def lbm_create(p, rho0, u0, wall_fields, workspace_ptr, workspace_bytes, stream_ptr):
    """u0: None or float64 [2, ny, nx] (u_x, u_y)."""
    out = _vp()
    _check(lib().lbm_create(ctypes.byref(p), _ptr(rho0), _ptr(u0), _ptr(wall_fields),
                            _vp(workspace_ptr), workspace_bytes, _vp(stream_ptr), ctypes.byref(out)))
    return out


def lbm_step(ctx, nsteps, residual=False):
    """Enqueues nsteps steps.  residual=True: passes residual_out (the call
    synchronises after every diagnostic pass and raises LbmError EUNSTABLE at
    the first non-finite one) and returns the latest residual."""
    if not residual:
        _check(lib().lbm_step(ctx, int(nsteps), None))
        return None
    r = ctypes.c_double()
    _check(lib().lbm_step(ctx, int(nsteps), ctypes.byref(r)))
    return r.value


def lbm_diagnostics(ctx, check=True):
    out = np.zeros(6)
    code = lib().lbm_diagnostics(ctx, _ptr(out))
    if check:
        _check(code)
    return out, code


def lbm_diagnostics_noalloc(ctx, check=True):
    """lbm_diagnostics with its partial sums in the library's static device
    array (no workspace scratch); see lbm.h."""
    out = np.zeros(6)
    code = lib().lbm_diagnostics_noalloc(ctx, _ptr(out))
    if check:
        _check(code)
    return out, code


def lbm_moments(ctx, n, want=(True, True, True)):
    arrs = [np.zeros(n) if w else None for w in want]
    tot = np.zeros(3)
    _check(lib().lbm_moments(ctx, *[_ptr(a) for a in arrs], _ptr(tot)))
    return arrs, tot


def lbm_contact_angle(ctx, iso, y_ref):
    out = np.zeros(4)
    code = lib().lbm_contact_angle(ctx, float(iso), float(y_ref), _ptr(out))
    if code == LBM_ENOFIT:
        return None
    _check(code)
    return out


def lbm_dynamic_angles(ctx, iso, y_ref):
    """(theta_A, theta_R, U, R_A, R_R, x_apex, y_apex, rho_L), or None when a
    fit has too few points; see lbm.h."""
    out = np.zeros(8)
    code = lib().lbm_dynamic_angles(ctx, float(iso), float(y_ref), _ptr(out))
    if code == LBM_ENOFIT:
        return None
    _check(code)
    return out


def lbm_slip_length(ctx):
    out = np.zeros(3)
    _check(lib().lbm_slip_length(ctx, _ptr(out)))
    return out


def lbm_get_state(ctx, n, q=9):
    f = np.zeros(q * n)
    _check(lib().lbm_get_state(ctx, _ptr(f)))
    return f


def lbm_set_state(ctx, f, step_index):
    f = _f64(f).ravel()
    _check(lib().lbm_set_state(ctx, _ptr(f), int(step_index)))


def lbm_step_index(ctx):
    return int(lib().lbm_step_index(ctx))


def lbm_destroy(ctx):
    if ctx:
        _check(lib().lbm_destroy(ctx))


def lbm_batch_workspace_bytes(ps):
    arr = (lbm_params * len(ps))(*ps)
    n = ctypes.c_size_t()
    _check(lib().lbm_batch_workspace_bytes(arr, len(ps), ctypes.byref(n)))
    return n.value


def lbm_batch_create(ps, rho0s, u0s, seg_rows, workspace_ptr, workspace_bytes, stream_ptr):
    n = len(ps)
    arr = (lbm_params * n)(*ps)

    def plist(lst):
        if lst is None:
            return None
        return (_dp * n)(*[_ptr(a) if a is not None else None for a in lst])

    out = _vp()
    _check(lib().lbm_batch_create(arr, n, plist(rho0s), plist(u0s), int(seg_rows),
                                  _vp(workspace_ptr), workspace_bytes, _vp(stream_ptr), ctypes.byref(out)))
    return out


def lbm_batch_step(b, nsteps, chunk=0):
    _check(lib().lbm_batch_step(b, int(nsteps), int(chunk)))


def lbm_batch_diagnostics(b, n, check=True):
    out = np.zeros(6 * n)
    code = lib().lbm_batch_diagnostics(b, _ptr(out))
    if check:
        _check(code)
    return out.reshape(n, 6), code


def lbm_batch_lattice(b, k):
    v = lib().lbm_batch_lattice(b, int(k))
    if not v:
        raise LbmError(LBM_EINVAL, lib().lbm_last_error(None).decode())
    return v


def lbm_batch_destroy(b):
    if b:
        _check(lib().lbm_batch_destroy(b))


def lbm_batch_attach_bytes(ctxs):
    arr = (_vp * len(ctxs))(*ctxs)
    n = ctypes.c_size_t()
    _check(lib().lbm_batch_attach_bytes(arr, len(ctxs), ctypes.byref(n)))
    return n.value


def lbm_batch_attach(ctxs, workspace_ptr, workspace_bytes, stream_ptr):
    arr = (_vp * len(ctxs))(*ctxs)
    out = _vp()
    _check(lib().lbm_batch_attach(arr, len(ctxs), _vp(workspace_ptr), workspace_bytes, _vp(stream_ptr),
                                  ctypes.byref(out)))
    return out


def lbm_tile_shapes():
    """[(waves, rows, strips), ...] of the step tile shapes, by shape id."""
    n = lib().lbm_tile_shapes(None, None, None, 0)
    w = np.zeros(n, dtype=np.int32)
    r = np.zeros(n, dtype=np.int32)
    s = np.zeros(n, dtype=np.int32)
    lib().lbm_tile_shapes(_iptr(w), _iptr(r), _iptr(s), n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(w, r, s)]


def lbm_set_tile_shape(ctx, shape):
    _check(lib().lbm_set_tile_shape(ctx, int(shape)))


def lbm_get_tile_shape(ctx):
    return int(lib().lbm_get_tile_shape(ctx))


def lbm_two_step_variants():
    """[(strips, rows, waves), ...] of the two-steps-per-pass variants."""
    n = lib().lbm_two_step_variants(None, None, None, 0)
    s = np.zeros(n, dtype=np.int32)
    r = np.zeros(n, dtype=np.int32)
    w = np.zeros(n, dtype=np.int32)
    lib().lbm_two_step_variants(_iptr(s), _iptr(r), _iptr(w), n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(s, r, w)]


def lbm_set_two_step(ctx, variant):
    _check(lib().lbm_set_two_step(ctx, int(variant)))


def lbm_get_two_step(ctx):
    return int(lib().lbm_get_two_step(ctx))


def lbm_tune_two_step(ctx, steps):
    """Returns (chosen variant or -1 for single steps, median ms per step of
    every variant followed by that of single steps)."""
    v = np.zeros(1, dtype=np.int32)
    ms = np.zeros(len(lbm_two_step_variants()) + 1)
    _check(lib().lbm_tune_two_step(ctx, int(steps), _iptr(v), _ptr(ms)))
    return int(v[0]), ms


def lbm_tune(ctx, steps):
    """Returns (chosen shape, median ms per step of every shape)."""
    shape = np.zeros(1, dtype=np.int32)
    ms = np.zeros(len(lbm_tile_shapes()))
    _check(lib().lbm_tune(ctx, int(steps), _iptr(shape), _ptr(ms)))
    return int(shape[0]), ms


def lbm_batch_set_tile_shapes(b, shapes):
    arr = None if shapes is None else np.ascontiguousarray(shapes, dtype=np.int32)
    _check(lib().lbm_batch_set_tile_shapes(b, None if arr is None else _iptr(arr)))


def lbm_batch_get_tile_shapes(b, n):
    out = np.zeros(n, dtype=np.int32)
    _check(lib().lbm_batch_get_tile_shapes(b, _iptr(out)))
    return out


def lbm_batch_tune(b, n, steps):
    """Returns (per-lattice shapes, median ms per step of each uniform shape
    and of the mixed assignment (NaN if not timed))."""
    shapes = np.zeros(n, dtype=np.int32)
    ms = np.zeros(len(lbm_tile_shapes()) + 1)
    _check(lib().lbm_batch_tune(b, int(steps), _iptr(shapes), _ptr(ms)))
    return shapes, ms


def lbm_batch_set_two_step(b, variant):
    _check(lib().lbm_batch_set_two_step(b, int(variant)))


def lbm_batch_get_two_step(b):
    return int(lib().lbm_batch_get_two_step(b))


def lbm_batch_tune_two_step(b, steps):
    """Returns (chosen variant or -1 for single steps, median ms per step of
    every variant followed by that of single steps), over the whole batch."""
    v = np.zeros(1, dtype=np.int32)
    ms = np.zeros(len(lbm_two_step_variants()) + 1)
    _check(lib().lbm_batch_tune_two_step(b, int(steps), _iptr(v), _ptr(ms)))
    return int(v[0]), ms


# ------------------------------------------------------------ conveniences
def _workspace(nbytes, device):
    import torch
    # over-allocate so the pointer can be aligned to 256 bytes
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = t.data_ptr()
    off = (-base) % 256
    return t, base + off


def _stream(device, stream):
    import torch
    if stream is not None:
        return stream.cuda_stream
    return torch.cuda.current_stream(device).cuda_stream


class Lattice:
    """One lattice on the GPU.  Fields are numpy float64 [ny, nx]."""

    def __init__(self, params, rho0, ux0=None, uy0=None, wall_fields=None, device="cuda:0", stream=None):
        self.p = params
        self.nx, self.ny = params.nx, params.ny
        self.n = self.nx * self.ny
        nbytes = lbm_workspace_bytes(params)
        self._ws, ptr = _workspace(nbytes, device)
        self.stream_ptr = _stream(device, stream)
        self.ctx = lbm_create(params, _f64(rho0), _u0(ux0, uy0), _f64(wall_fields), ptr, nbytes,
                              self.stream_ptr)
        self.workspace_bytes = nbytes

    def step(self, nsteps=1, residual=False):
        """Advance nsteps; residual=True returns the latest diagnostic
        residual and raises LbmError EUNSTABLE on non-finite values (see
        lbm_step)."""
        return lbm_step(self.ctx, nsteps, residual)

    @property
    def last_error(self):
        return lbm_last_error(self.ctx)

    def diagnostics(self, check=True):
        return lbm_diagnostics(self.ctx, check)[0]

    def moments(self):
        (rho, ux, uy), tot = lbm_moments(self.ctx, self.n)
        shp = (self.ny, self.nx)
        return rho.reshape(shp), ux.reshape(shp), uy.reshape(shp), tot

    def contact_angle(self, iso=1.07, y_ref=0.0):
        return lbm_contact_angle(self.ctx, iso, y_ref)

    def dynamic_angles(self, iso=1.07, y_ref=0.0):
        return lbm_dynamic_angles(self.ctx, iso, y_ref)

    def slip_length(self):
        return lbm_slip_length(self.ctx)

    def get_state(self):
        """Populations as float64 [Q, ny, nx] (post-streaming)."""
        q = nq(self.p)
        return lbm_get_state(self.ctx, self.n, q).reshape(q, self.ny, self.nx)

    def set_state(self, f, step_index=0):
        f = np.asarray(f)
        if f.size != nq(self.p) * self.n:
            raise ValueError(f"state must hold {nq(self.p)} x {self.ny} x {self.nx} values")
        lbm_set_state(self.ctx, f, step_index)

    @property
    def step_index(self):
        return lbm_step_index(self.ctx)

    @property
    def tile_shape(self):
        """D2Q9: index into lbm_tile_shapes(); D2Q21: step variant (0 two-row
        tiles, 1 marching, binary32 only, 2 one-row tiles).  Every choice
        computes bitwise the same update."""
        return lbm_get_tile_shape(self.ctx)

    @tile_shape.setter
    def tile_shape(self, shape):
        lbm_set_tile_shape(self.ctx, shape)

    @property
    def two_step(self):
        """Two-steps-per-pass variant (index into lbm_two_step_variants()),
        -1 for single steps.  Bitwise the same fields either way."""
        return lbm_get_two_step(self.ctx)

    @two_step.setter
    def two_step(self, variant):
        lbm_set_two_step(self.ctx, variant)

    def tune(self, steps=10):
        """Autotune the tile shape (advances the lattice; see lbm_tune)."""
        return lbm_tune(self.ctx, steps)

    def tune_two_step(self, steps=10):
        """Choose between single steps and two steps per pass (advances the
        lattice; see lbm_tune_two_step)."""
        return lbm_tune_two_step(self.ctx, steps)

    def close(self):
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Attached:
    """A batch over existing Lattice objects (all on one non-default stream):
    one launch per time step for all of them; closing hands them back."""

    def __init__(self, lattices, device="cuda:0"):
        self.lattices = list(lattices)
        ctxs = [L.ctx for L in self.lattices]
        streams = {L.stream_ptr for L in self.lattices}
        if len(streams) != 1:
            raise ValueError("attached lattices must share one stream")
        self.stream_ptr = streams.pop()
        nbytes = lbm_batch_attach_bytes(ctxs)
        self._ws, ptr = _workspace(nbytes, device)
        self.b = lbm_batch_attach(ctxs, ptr, nbytes, self.stream_ptr)
        self.n = len(ctxs)

    def step(self, nsteps, chunk=0):
        lbm_batch_step(self.b, nsteps, chunk)

    def diagnostics(self, check=True):
        return lbm_batch_diagnostics(self.b, self.n, check)

    @property
    def tile_shapes(self):
        return lbm_batch_get_tile_shapes(self.b, self.n)

    @tile_shapes.setter
    def tile_shapes(self, shapes):
        lbm_batch_set_tile_shapes(self.b, shapes)

    def tune(self, steps=10):
        return lbm_batch_tune(self.b, self.n, steps)

    @property
    def two_step(self):
        """Two-steps-per-pass variant of the batch, -1 for single steps."""
        return lbm_batch_get_two_step(self.b)

    @two_step.setter
    def two_step(self, variant):
        lbm_batch_set_two_step(self.b, variant)

    def tune_two_step(self, steps=5):
        """Choose between single steps and two steps per pass for the whole
        batch (advances every lattice; see lbm_batch_tune_two_step)."""
        return lbm_batch_tune_two_step(self.b, steps)

    def close(self):
        if self.b:
            lbm_batch_destroy(self.b)
            self.b = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class View:
    """A lattice inside a Batch (moments, angle, slip, state, diagnostics)."""

    def __init__(self, batch, k, params):
        self.ctx = lbm_batch_lattice(batch.b, k)
        self.p = params
        self.nx, self.ny = params.nx, params.ny
        self.n = self.nx * self.ny

    moments = Lattice.moments
    contact_angle = Lattice.contact_angle
    slip_length = Lattice.slip_length
    get_state = Lattice.get_state
    diagnostics = Lattice.diagnostics


class Batch:
    """Many independent F32 lattices advanced by one launch per time step."""

    def __init__(self, params_list, rho0s, ux0s=None, uy0s=None, seg_rows=0, device="cuda:0", stream=None):
        self.ps = list(params_list)
        for p in self.ps:
            p.seg_rows = seg_rows
        nbytes = lbm_batch_workspace_bytes(self.ps)
        self._ws, ptr = _workspace(nbytes, device)
        if stream is None:
            # graph capture needs a stream other than the legacy default one
            import torch
            torch.cuda.synchronize(device)
            stream = torch.cuda.Stream(device)
        self._stream_obj = stream
        self.stream_ptr = _stream(device, stream)
        rho0s = [_f64(r) for r in rho0s]
        u0s = None
        if ux0s is not None or uy0s is not None:
            u0s = [_u0(a, b) for a, b in zip(ux0s, uy0s)]
        self.b = lbm_batch_create(self.ps, rho0s, u0s, seg_rows, ptr, nbytes, self.stream_ptr)
        self.workspace_bytes = nbytes
        self.n = len(self.ps)

    def step(self, nsteps, chunk=0):
        lbm_batch_step(self.b, nsteps, chunk)

    def diagnostics(self, check=True):
        return lbm_batch_diagnostics(self.b, self.n, check)[0]

    tile_shapes = Attached.tile_shapes
    tune = Attached.tune
    two_step = Attached.two_step
    tune_two_step = Attached.tune_two_step

    def lattice(self, k):
        return View(self, k, self.ps[k])

    def close(self):
        if self.b:
            lbm_batch_destroy(self.b)
            self.b = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
