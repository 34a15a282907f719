"""ctypes binding of libpfch (include/pfch.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device arrays are torch tensors (float64, contiguous, on the GPU); their
``data_ptr()`` and the current torch stream are handed to the C ABI.
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfch.so")

PFCH_OK = 0
PFCH_E_INVAL = -1
PFCH_E_NOMEM = -2
PFCH_E_HIP = -3
PFCH_E_NOCONV = -4
PFCH_E_NONFINITE = -5
PFCH_E_PRECOND = -6
PFCH_E_UNSUPPORTED = -7
PFCH_E_INTERNAL = -8
PFCH_E_SCRATCH = -9

PFC, FCH = 0, 1
BDF2, MP, LBDF2, LMP = 0, 1, 2, 3

PAPER_ETAS = tuple(math.sqrt(v) for v in (0.1, 0.575, 1.05, 1.525, 2.0))

EST_AUTO, EST_AM3, EST_MIDAB2 = 0, 1, 2

EXPORTED = (
    "pfch_validate_desc", "pfch_create", "pfch_set_state", "pfch_get_state",
    "pfch_step", "pfch_solve", "pfch_set_stats_detail", "pfch_time_kernels",
    "pfch_get_launch_config", "pfch_destroy", "pfch_time_kernels_events",
    "pfch_strerror", "pfch_version",
    "pfch_fno_num_params", "pfch_fno_create", "pfch_fno_init_params", "pfch_fno_set_params",
    "pfch_fno_get_params", "pfch_fno_forward", "pfch_fno_grad", "pfch_fno_adam_step",
    "pfch_fno_prepare", "pfch_fno_destroy", "pfch_set_fno", "pfch_get_plan", "pfch_set_plan",
    "pfch_step_adaptive", "pfch_rhs", "pfch_fno_num_params_3d", "pfch_fno_create_3d",
    "pfch_stop_status", "pfch_rhs_noalloc", "pfch_fno_prepare_resampled", "pfch_time_group",
)


# codes that are errors of the call, not per-instance solver outcomes
_HARD_ERRORS = (PFCH_E_INVAL, PFCH_E_NOMEM, PFCH_E_HIP, PFCH_E_UNSUPPORTED, PFCH_E_INTERNAL)


class InstanceDesc(ctypes.Structure):
    _fields_ = [
        ("len", ctypes.c_double * 3),
        ("eps", ctypes.c_double), ("eta1", ctypes.c_double), ("eta2", ctypes.c_double),
        ("tau", ctypes.c_double), ("mobility", ctypes.c_double),
        ("s", ctypes.c_double), ("tol", ctypes.c_double), ("theta_l", ctypes.c_double),
        ("eta", ctypes.c_double * 8),
        ("model", ctypes.c_int32), ("scheme", ctypes.c_int32), ("ndim", ctypes.c_int32),
        ("n_eta", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("guess", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("reserved", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("dnorm_inf", ctypes.c_double),
        ("beta", ctypes.c_double * 4),
        ("mass", ctypes.c_double),
        ("rnorm_inf", ctypes.c_double),
        ("gain", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("fft_pairs", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("guess", ctypes.c_int32),
    ]

    def as_dict(self):
        return dict(iters=self.iters, status=self.status, dnorm=self.dnorm_inf,
                    betas=tuple(self.beta), mass=self.mass, fft_pairs=self.fft_pairs,
                    guess=self.guess, rnorm=self.rnorm_inf, gain=self.gain)


class AdaptDesc(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double), ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("estimator", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class AdaptResult(ctypes.Structure):
    _fields_ = [
        ("dt_try", ctypes.c_double), ("dt", ctypes.c_double), ("err", ctypes.c_double),
        ("accepted", ctypes.c_int32), ("estimator", ctypes.c_int32),
        ("solve", Stats),
    ]

    def as_dict(self):
        return dict(dt=self.dt, err=self.err, accepted=bool(self.accepted),
                    estimator={EST_AM3: "am3", EST_MIDAB2: "midab2"}.get(self.estimator),
                    dt_next=self.dt_try, solve=self.solve.as_dict())


class PfchError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib():
    """Load libpfch.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2204_07247_amd.build`")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so that both share one runtime and one device context
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.pfch_validate_desc.argtypes = [ctypes.POINTER(InstanceDesc)]
        L.pfch_create.argtypes = [ctypes.POINTER(InstanceDesc), i32, vp, ctypes.POINTER(vp)]
        L.pfch_set_state.argtypes = [vp, i32, vp, vp, dbl, dbl, i32]
        L.pfch_get_state.argtypes = [vp, i32, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(i32)]
        L.pfch_step.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(Stats)]
        L.pfch_solve.argtypes = [vp, i32, dbl, dbl, dbl, vp, vp, vp, ctypes.POINTER(Stats)]
        L.pfch_set_stats_detail.argtypes = [vp, i32]
        L.pfch_time_kernels.argtypes = [vp, dbl, i32, ctypes.POINTER(dbl)]
        L.pfch_time_kernels_events.argtypes = [vp, dbl, i32, ctypes.POINTER(dbl)]
        L.pfch_time_kernels_events.restype = ctypes.c_int
        L.pfch_time_group.argtypes = [vp, i32, dbl, i32, ctypes.POINTER(dbl)]
        L.pfch_time_group.restype = ctypes.c_int
        L.pfch_get_launch_config.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
        L.pfch_destroy.argtypes = [vp]
        L.pfch_destroy.restype = None
        L.pfch_strerror.argtypes = [ctypes.c_int]
        L.pfch_strerror.restype = ctypes.c_char_p
        L.pfch_version.argtypes = []
        fp = ctypes.c_void_p
        L.pfch_fno_num_params.argtypes = [i32, i32, i32]
        L.pfch_fno_num_params.restype = ctypes.c_int64
        L.pfch_fno_create.argtypes = [i32, i32, i32, i32, i32, i32, vp, ctypes.POINTER(vp)]
        L.pfch_fno_num_params_3d.argtypes = [i32, i32, i32]
        L.pfch_fno_num_params_3d.restype = ctypes.c_int64
        L.pfch_fno_create_3d.argtypes = [i32, i32, i32, i32, i32, i32, i32, vp, ctypes.POINTER(vp)]
        L.pfch_fno_init_params.argtypes = [fp, ctypes.c_uint64]
        L.pfch_fno_set_params.argtypes = [fp, vp, ctypes.c_int64]
        L.pfch_fno_get_params.argtypes = [fp, vp, ctypes.c_int64]
        L.pfch_fno_forward.argtypes = [fp, vp, vp, i32]
        L.pfch_fno_grad.argtypes = [fp, vp, vp, i32, vp, ctypes.POINTER(dbl)]
        L.pfch_fno_adam_step.argtypes = [fp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, i32]
        L.pfch_fno_prepare.argtypes = [fp, vp, vp, vp, dbl, ctypes.POINTER(dbl), vp, vp]
        L.pfch_fno_prepare_resampled.argtypes = [fp, i32, i32, vp, vp, vp, dbl, ctypes.POINTER(dbl), vp, vp]
        L.pfch_fno_destroy.argtypes = [fp]
        L.pfch_fno_destroy.restype = None
        L.pfch_set_fno.argtypes = [vp, i32, fp, ctypes.POINTER(dbl)]
        L.pfch_get_plan.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.pfch_set_plan.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.pfch_get_plan.restype = ctypes.c_int
        L.pfch_step_adaptive.argtypes = [vp, ctypes.POINTER(AdaptDesc), ctypes.POINTER(AdaptResult)]
        L.pfch_step_adaptive.restype = ctypes.c_int
        L.pfch_rhs.argtypes = [vp, i32, vp, vp]
        L.pfch_rhs.restype = ctypes.c_int
        L.pfch_rhs_noalloc.argtypes = [vp, i32, vp, vp]
        L.pfch_rhs_noalloc.restype = ctypes.c_int
        L.pfch_set_plan.restype = ctypes.c_int
        L.pfch_stop_status.argtypes = [i32, i32, ctypes.c_uint64, i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(dbl)]
        L.pfch_stop_status.restype = ctypes.c_int
        for name in ("pfch_fno_create", "pfch_fno_create_3d", "pfch_fno_init_params", "pfch_fno_set_params",
                     "pfch_fno_get_params", "pfch_fno_forward", "pfch_fno_grad",
                     "pfch_fno_adam_step", "pfch_fno_prepare", "pfch_set_fno", "pfch_fno_prepare_resampled"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("pfch_validate_desc", "pfch_create", "pfch_set_state", "pfch_get_state",
                     "pfch_step", "pfch_solve", "pfch_set_stats_detail", "pfch_time_kernels",
                     "pfch_get_launch_config", "pfch_version"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code):
    return lib().pfch_strerror(int(code)).decode()


def stop_status(stop_iter, flags, norm_bits, max_iter):
    """The host's decision on a stop record (pfch_stop_status): (code, iters, dnorm)."""
    it = ctypes.c_int32()
    dn = ctypes.c_double()
    rc = lib().pfch_stop_status(int(stop_iter), int(flags), int(norm_bits), int(max_iter),
                                ctypes.byref(it), ctypes.byref(dn))
    return rc, it.value, dn.value


def make_desc(model, scheme, shape, lengths, eps, eta1=0.0, eta2=0.0, tau=0.0,
              mobility=1.0, s=0.9, etas=PAPER_ETAS, tol=1e-10, max_iter=1000,
              theta_l=1.0, guess=0):
    """Descriptor from plain values.  ``shape``/``lengths`` are in array
    order ((Ny, Nx) in 2D); the C struct stores them x first."""
    d = InstanceDesc()
    nd = len(shape)
    for a in range(nd):
        d.n[a] = int(shape[nd - 1 - a])
        d.len[a] = float(lengths[nd - 1 - a])
    d.ndim = nd
    d.model = {"pfc": PFC, "fch": FCH}.get(model, model)
    d.scheme = {"bdf2": BDF2, "mp": MP, "lbdf2": LBDF2, "lmp": LMP}.get(scheme, scheme)
    d.eps, d.eta1, d.eta2, d.tau, d.mobility = eps, eta1, eta2, tau, mobility
    d.s, d.tol, d.theta_l = s, tol, theta_l
    etas = tuple(etas)  # () selects plain preconditioned gradient descent (no momentum)
    d.n_eta = len(etas)
    for i, e in enumerate(etas):
        d.eta[i] = e
    d.max_iter = int(max_iter)
    d.guess = int(guess)
    d.reserved = 0
    return d


def validate_desc(desc):
    return lib().pfch_validate_desc(ctypes.byref(desc))


def _ptr(t, dtype="float64"):
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous GPU tensor")
    import torch
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"expected {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _fptr(t):
    return _ptr(t, "float32")


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _timing(out, chained):
    if out[2] == 0.0 and out[3] == 0.0:
        d = dict(col_us=out[0], row_us=out[1])
    else:
        d = dict(yfwd_us=out[0], z_us=out[1], yinv_us=out[2], row_us=out[3])
    if chained:
        d["iteration_us"] = out[4]
    return d


class Context:
    """A set of instances that advance together (pfch_create ... pfch_destroy)."""

    def __init__(self, descs, stream=None):
        L = lib()
        if isinstance(descs, InstanceDesc):
            descs = [descs]
        self.n = len(descs)
        arr = (InstanceDesc * self.n)(*descs)
        self._descs = arr
        h = ctypes.c_void_p()
        s = _stream_handle() if stream is None else ctypes.c_void_p(stream)
        rc = L.pfch_create(arr, self.n, s, ctypes.byref(h))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pfch_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stats_detail(self, detail):
        rc = lib().pfch_set_stats_detail(self._h, int(detail))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_set_stats_detail")

    def time_kernels(self, dt, reps, events=False):
        """Average microseconds per launch of instance 0's iteration kernels:
        HIP events on every launch of `reps` solves (default), or HIP events
        around `reps` back-to-back launches of each kernel (events=True).
        2D {col_us, row_us}; 3D {yfwd_us, z_us, yinv_us, row_us}; with the
        solve's timing also iteration_us, the time per iteration of the
        chain of launches without per-launch events."""
        out = (ctypes.c_double * 5)()
        fn = lib().pfch_time_kernels_events if events else lib().pfch_time_kernels
        rc = fn(self._h, float(dt), int(reps), out)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_time_kernels")
        return _timing(out, not events)

    def time_group(self, inst, dt, reps):
        """Average microseconds per grouped launch of the iteration kernels of
        instance `inst`'s group (pfch_time_group); keys as time_kernels."""
        out = (ctypes.c_double * 5)()
        rc = lib().pfch_time_group(self._h, int(inst), float(dt), int(reps), out)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_time_group")
        return _timing(out, True)

    def launch_config(self, inst=0):
        out = (ctypes.c_int64 * 6)()
        rc = lib().pfch_get_launch_config(self._h, inst, out)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_get_launch_config")
        return dict(row_grid=out[0], row_block=out[1], row_lds=out[2], col_grid=out[3],
                    col_block=out[4], col_lds=out[5])

    def set_state(self, inst, u_n, u_nm1=None, t=0.0, dt_prev=0.0, step_index=0):
        rc = lib().pfch_set_state(self._h, inst, _ptr(u_n), _ptr(u_nm1), float(t),
                                  float(dt_prev), int(step_index))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_set_state")

    def get_state(self, inst, u_n=None, u_nm1=None):
        t = ctypes.c_double()
        dtp = ctypes.c_double()
        n = ctypes.c_int32()
        rc = lib().pfch_get_state(self._h, inst, _ptr(u_n), _ptr(u_nm1), ctypes.byref(t),
                                  ctypes.byref(dtp), ctypes.byref(n))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_get_state")
        return t.value, dtp.value, n.value

    def step(self, dt, stats=True):
        """One step of every instance; returns (code, [stats dict per instance])."""
        if isinstance(dt, (int, float)):
            dt = [float(dt)] * self.n
        dts = (ctypes.c_double * self.n)(*dt)
        st = (Stats * self.n)() if stats else None
        rc = lib().pfch_step(self._h, dts, st)
        if rc in _HARD_ERRORS:
            raise PfchError(rc, "pfch_step")
        return rc, ([s.as_dict() for s in st] if stats else None)

    def step_adaptive(self, dt_try, tol, dt_min, dt_max, estimator=EST_AUTO):
        """One attempt of adaptive stepping for every instance (pfch_step_adaptive).
        ``dt_try``: tentative size(s).  Returns (code, [result dict per
        instance]); each result's ``dt_next`` is the next tentative size."""
        if isinstance(dt_try, (int, float)):
            dt_try = [float(dt_try)] * self.n
        ad = AdaptDesc(float(tol), float(dt_min), float(dt_max),
                       {"auto": EST_AUTO, "am3": EST_AM3, "midab2": EST_MIDAB2}.get(estimator, estimator), 0)
        res = (AdaptResult * self.n)()
        for i, d in enumerate(dt_try):
            res[i].dt_try = float(d)
        rc = lib().pfch_step_adaptive(self._h, ctypes.byref(ad), res)
        if rc in _HARD_ERRORS:
            raise PfchError(rc, "pfch_step_adaptive")
        return rc, [r.as_dict() for r in res]

    def rhs(self, inst, v, out):
        """out = M Delta mu(v) for instance ``inst``'s model and grid."""
        rc = lib().pfch_rhs(self._h, int(inst), _ptr(v), _ptr(out))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_rhs")

    def rhs_noalloc(self, inst, v, out):
        """pfch_rhs_noalloc: out = M Delta mu(v) in the library's static
        scratch, with no allocation or synchronisation; returns the code."""
        return lib().pfch_rhs_noalloc(self._h, int(inst), _ptr(v), _ptr(out))

    def plan(self, inst=0):
        """Iteration-kernel plans of the instance's group (see pfch_get_plan)."""
        out = (ctypes.c_int32 * 37)()
        rc = lib().pfch_get_plan(self._h, inst, out)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_get_plan")
        rad = lambda v: [r for r in v if r > 1]
        return dict(row_alt=out[0], row_teams=out[1], col_alt=out[2], col_cb=out[3],
                    y_alt=out[4], y_cb=out[5], z_alt=out[6], z_kyb=out[7],
                    n_row_alts=out[8], n_col_alts=out[9], n_y_alts=out[10], n_z_alts=out[11],
                    row_radices=rad(out[12:20]), col_radices=rad(out[20:28]),
                    z_radices=rad(out[28:36]))

    def set_plan(self, inst, row_alt, teams, col_alt=-1, cb=1, y_alt=-1, y_cb=1, z_alt=-1,
                 z_kyb=1):
        ch = (ctypes.c_int32 * 9)(row_alt, teams, col_alt, cb, y_alt, y_cb, z_alt, z_kyb, 0)
        rc = lib().pfch_set_plan(self._h, inst, ch)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_set_plan")

    def set_fno(self, inst, fno, norm=None):
        """Attach an Fno (None detaches) to instance `inst` with
        norm = (mu, su, sd, so)."""
        nrm = (ctypes.c_double * 4)(*(norm if norm is not None else (0.0, 1.0, 1.0, 1.0)))
        self._fno_refs = getattr(self, "_fno_refs", {})
        self._fno_refs[inst] = fno
        rc = lib().pfch_set_fno(self._h, inst, fno._h if fno is not None else None, nrm)
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_set_fno")

    def solve(self, inst, a, b, c, u_n, u_nm1, x):
        st = Stats()
        rc = lib().pfch_solve(self._h, inst, float(a), float(b), float(c), _ptr(u_n),
                              _ptr(u_nm1), _ptr(x), ctypes.byref(st))
        if rc in _HARD_ERRORS:
            raise PfchError(rc, "pfch_solve")
        return rc, st.as_dict()


def fno_num_params(width, modes, layers, ndim=2):
    f = lib().pfch_fno_num_params_3d if ndim == 3 else lib().pfch_fno_num_params
    return int(f(width, modes, layers))


class Fno:
    """Float32 Fourier neural operator on the GPU (pfch_fno_* entry points).
    `shape` is the grid, (Ny, Nx) or (Nz, Ny, Nx).  Arrays are contiguous
    float32 GPU tensors: x [B, 2, *shape], y/t [B, *shape], parameters [n]."""

    def __init__(self, width, modes, layers, *shape, max_batch=1, stream=None):
        if len(shape) not in (2, 3):
            raise ValueError("Fno grid must be (Ny, Nx) or (Nz, Ny, Nx)")
        L = lib()
        h = ctypes.c_void_p()
        s = _stream_handle() if stream is None else ctypes.c_void_p(stream)
        if len(shape) == 3:
            rc = L.pfch_fno_create_3d(width, modes, layers, *shape, max_batch, s, ctypes.byref(h))
        else:
            rc = L.pfch_fno_create(width, modes, layers, *shape, max_batch, s, ctypes.byref(h))
        if rc != PFCH_OK:
            raise PfchError(rc, "pfch_fno_create")
        self._h = h
        self.width, self.modes, self.layers = width, modes, layers
        self.shape = tuple(int(n) for n in shape)
        self.max_batch = max_batch
        self.n_params = fno_num_params(width, modes, layers, len(shape))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pfch_fno_destroy(self._h)
        self._h = None

    __del__ = close

    def _check(self, rc, where):
        if rc != PFCH_OK:
            raise PfchError(rc, where)

    def init_params(self, seed=0):
        self._check(lib().pfch_fno_init_params(self._h, int(seed)), "pfch_fno_init_params")

    def set_params(self, theta):
        self._check(lib().pfch_fno_set_params(self._h, _fptr(theta), theta.numel()),
                    "pfch_fno_set_params")

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(lib().pfch_fno_get_params(self._h, _fptr(out), out.numel()), "pfch_fno_get_params")
        return out

    def forward(self, x):
        import torch
        b = x.shape[0]
        y = torch.empty((b,) + tuple(self.shape), dtype=torch.float32, device=x.device)
        self._check(lib().pfch_fno_forward(self._h, _fptr(x), _fptr(y), b), "pfch_fno_forward")
        return y

    def grad(self, x, t, want_grad=True, want_loss=True):
        """(loss or None, gradient tensor or None)."""
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device) if want_grad else None
        loss = ctypes.c_double()
        self._check(lib().pfch_fno_grad(self._h, _fptr(x), _fptr(t), x.shape[0],
                                        _fptr(g) if g is not None else None,
                                        ctypes.byref(loss) if want_loss else None), "pfch_fno_grad")
        return (loss.value if want_loss else None), g

    def adam_step(self, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib().pfch_fno_adam_step(self._h, lr, beta1, beta2, eps, int(step)),
                    "pfch_fno_adam_step")

    def prepare(self, u_nm1, u_n, u_np1, rho, norm, x, t=None):
        """Fill x [2, *shape] (and t [*shape]) of one sample from float64
        fields; fields on a finer 2D grid than the network's are resampled
        to it (pfch_fno_prepare_resampled)."""
        nrm = (ctypes.c_double * 4)(*norm)
        if tuple(u_n.shape) != self.shape:
            ny, nx = u_n.shape
            self._check(lib().pfch_fno_prepare_resampled(self._h, int(ny), int(nx), _ptr(u_nm1), _ptr(u_n),
                                                         _ptr(u_np1), float(rho), nrm, _fptr(x), _fptr(t)),
                        "pfch_fno_prepare_resampled")
            return
        self._check(lib().pfch_fno_prepare(self._h, _ptr(u_nm1), _ptr(u_n), _ptr(u_np1), float(rho),
                                           nrm, _fptr(x), _fptr(t)), "pfch_fno_prepare")
