"""Python binding of libelwh.so (ctypes).  Argument marshalling only: every
step of the filter and the Krylov solve runs in the library's HIP kernels.

torch is imported before the library is loaded, so libelwh binds to the HIP
runtime torch already loaded, and torch supplies device memory and streams.
If the library is not built, importing this module raises: there is no CPU
fallback on the product path.
"""

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede loading the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelwh.so")

OK, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_UNSTABLE, ERR_NOT_CONVERGED, ERR_BREAKDOWN = range(7)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_ALLOC", "ERR_HIP", "ERR_UNSTABLE", "ERR_NOT_CONVERGED", "ERR_BREAKDOWN"]
BC_DIRICHLET, BC_TRACTION_FREE, BC_IMPEDANCE = 0, 1, 2
FP64, FP32_STEP = 0, 1
KRYLOV_CG, KRYLOV_GMRES, KRYLOV_CR, KRYLOV_MINRES = 0, 1, 2, 3
SCHEME_CORRECTED, SCHEME_STANDARD, SCHEME_MODIFIED = 0, 1, 2
FALLBACK_NONE, FALLBACK_CR, FALLBACK_MINRES = 0, 1, 2

EXPORTED = [
    "elwh_default_opts", "elwh_plan", "elwh_create", "elwh_plan_mapped", "elwh_create_mapped",
    "elwh_plan_mapped3", "elwh_create_mapped3",
    "elwh_filter_diagnostics", "elwh_destroy", "elwh_query", "elwh_last_error",
    "elwh_apply_filter", "elwh_apply_A", "elwh_solve", "elwh_cg_begin", "elwh_cg_iterate",
    "elwh_apply_filter2", "elwh_apply_A2", "elwh_solve2",
    "elwh_cg_result", "elwh_dot_M", "elwh_profile_enable", "elwh_profile_read",
    "elwh_set_tile", "elwh_get_tile", "elwh_autotune",
    "elwh_batch_create", "elwh_batch_solve", "elwh_batch_set_graph", "elwh_batch_info", "elwh_batch_stats",
    "elwh_batch_last_error", "elwh_batch_destroy",
    "elwh_ws_create", "elwh_ws_destroy", "elwh_ws_last_error", "elwh_ws_num_params", "elwh_ws_params",
    "elwh_ws_forward", "elwh_ws_loss_grad", "elwh_ws_train_step", "elwh_ws_features", "elwh_ws_from_field",
    "elwh_ws_predict", "elwh_ws_normalize", "elwh_dot_M_noalloc", "elwh_stream_triad",
]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("len", ctypes.c_double * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("cfl", ctypes.c_double), ("nt", ctypes.c_int), ("periods", ctypes.c_int),
                ("prec", ctypes.c_int), ("krylov", ctypes.c_int), ("gmres_m", ctypes.c_int),
                ("scheme", ctypes.c_int), ("compensated", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("stream", ctypes.c_void_p), ("autotune", ctypes.c_int),
                ("fuse", ctypes.c_int), ("scale_x0", ctypes.c_int), ("cr_fallback", ctypes.c_int),
                ("fp64_fallback", ctypes.c_int), ("fp32_switch", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("nt", ctypes.c_int), ("napply", ctypes.c_int),
                ("dt", ctypes.c_double), ("c", ctypes.c_double), ("lambda_bound", ctypes.c_double),
                ("relres", ctypes.c_double), ("relres_fp64", ctypes.c_double), ("cond_est", ctypes.c_double),
                ("cr_iters", ctypes.c_int), ("fp64_iters", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FilterDiag(ctypes.Structure):
    _fields_ = [("r_star", ctypes.c_double), ("gap", ctypes.c_double), ("beta_max", ctypes.c_double),
                ("r_max", ctypes.c_double), ("lambda_lo", ctypes.c_double), ("lambda_hi", ctypes.c_double)]


class ElwhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2205_12344_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    lib.elwh_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.elwh_default_opts.restype = None
    lib.elwh_plan.argtypes = [ctypes.POINTER(Grid), P, P, P, D, ctypes.POINTER(I), ctypes.POINTER(Opts),
                              ctypes.POINTER(Info)]
    lib.elwh_create.argtypes = [ctypes.POINTER(Grid), P, P, P, D, ctypes.POINTER(I), ctypes.POINTER(Opts),
                                ctypes.POINTER(P)]
    lib.elwh_create_mapped.argtypes = [ctypes.POINTER(Grid), P, P, P, P, P, D, ctypes.POINTER(I),
                                       ctypes.POINTER(Opts), ctypes.POINTER(P)]
    lib.elwh_plan_mapped.argtypes = [ctypes.POINTER(Grid), P, P, P, P, P, D, ctypes.POINTER(I),
                                     ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.elwh_create_mapped3.argtypes = [ctypes.POINTER(Grid), P, P, P, P, P, P, D, ctypes.POINTER(I),
                                        ctypes.POINTER(Opts), ctypes.POINTER(P)]
    lib.elwh_plan_mapped3.argtypes = [ctypes.POINTER(Grid), P, P, P, P, P, P, D, ctypes.POINTER(I),
                                      ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.elwh_filter_diagnostics.argtypes = [I, I, D, I, ctypes.POINTER(FilterDiag)]
    lib.elwh_destroy.argtypes = [P]
    lib.elwh_destroy.restype = None
    lib.elwh_query.argtypes = [P, ctypes.POINTER(Info)]
    lib.elwh_last_error.argtypes = [P]
    lib.elwh_last_error.restype = ctypes.c_char_p
    lib.elwh_apply_filter.argtypes = [P, P, P, P]
    lib.elwh_apply_A.argtypes = [P, P, P]
    lib.elwh_solve.argtypes = [P, P, P, D, I, P, ctypes.POINTER(Info)]
    lib.elwh_apply_filter2.argtypes = [P, P, P, P, P, P]
    lib.elwh_apply_A2.argtypes = [P, P, P, P, P]
    lib.elwh_solve2.argtypes = [P, P, P, P, D, I, P, P, ctypes.POINTER(Info)]
    lib.elwh_cg_begin.argtypes = [P, P, P]
    lib.elwh_cg_iterate.argtypes = [P, I, D, ctypes.POINTER(D)]
    lib.elwh_cg_result.argtypes = [P, P, ctypes.POINTER(Info)]
    lib.elwh_dot_M.argtypes = [P, P, P, ctypes.POINTER(D)]
    lib.elwh_stream_triad.argtypes = [P, P, P, D, ctypes.c_longlong, P]
    lib.elwh_dot_M_noalloc.argtypes = [ctypes.POINTER(Grid), P, ctypes.POINTER(I), P, P, P, ctypes.POINTER(D)]
    lib.elwh_set_tile.argtypes = [P, I, I, I]
    lib.elwh_get_tile.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.elwh_autotune.argtypes = [P, I, I, ctypes.POINTER(D)]
    PP = ctypes.POINTER(P)
    lib.elwh_batch_create.argtypes = [I, ctypes.POINTER(Grid), PP, PP, PP, ctypes.POINTER(D), ctypes.POINTER(I),
                                      ctypes.POINTER(Opts), ctypes.POINTER(P)]
    lib.elwh_batch_solve.argtypes = [P, PP, PP, D, I, PP, ctypes.POINTER(Info)]
    lib.elwh_batch_set_graph.argtypes = [P, I]
    lib.elwh_batch_info.argtypes = [P, I, ctypes.POINTER(Info)]
    lib.elwh_batch_stats.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(I),
                                     ctypes.POINTER(I)]
    lib.elwh_batch_last_error.argtypes = [P]
    lib.elwh_batch_last_error.restype = ctypes.c_char_p
    lib.elwh_batch_destroy.argtypes = [P]
    lib.elwh_batch_destroy.restype = None
    F = ctypes.POINTER(ctypes.c_float)
    lib.elwh_ws_create.argtypes = [I, I, I, ctypes.c_ulonglong, P, ctypes.POINTER(P)]
    lib.elwh_ws_destroy.argtypes = [P]
    lib.elwh_ws_destroy.restype = None
    lib.elwh_ws_last_error.argtypes = [P]
    lib.elwh_ws_last_error.restype = ctypes.c_char_p
    lib.elwh_ws_num_params.argtypes = [P]
    lib.elwh_ws_num_params.restype = ctypes.c_longlong
    lib.elwh_ws_params.argtypes = [P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.elwh_ws_forward.argtypes = [P, I, P, P]
    lib.elwh_ws_loss_grad.argtypes = [P, I, P, P, P, F, P]
    lib.elwh_ws_train_step.argtypes = [P, I, P, P, P, ctypes.c_float, F]
    lib.elwh_ws_features.argtypes = [P, I, I, PP, PP, PP, PP, P, P, P]
    lib.elwh_ws_from_field.argtypes = [P, I, I, PP, PP, P, P]
    lib.elwh_ws_predict.argtypes = [P, I, I, P, PP, P, PP]
    lib.elwh_ws_normalize.argtypes = [P, I, P, P]
    lib.elwh_profile_enable.argtypes = [P, I]
    lib.elwh_profile_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(D),
                                      ctypes.POINTER(I)]
    for name in EXPORTED:
        if name not in ("elwh_default_opts", "elwh_destroy", "elwh_last_error", "elwh_batch_last_error",
                        "elwh_batch_destroy", "elwh_ws_destroy", "elwh_ws_last_error", "elwh_ws_num_params"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def default_opts(**kw):
    o = Opts()
    lib.elwh_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "stream":
            v = ctypes.c_void_p(v)
        setattr(o, k, v)
    return o


def make_grid(dim, n, length=None):
    g = Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a]) if a < dim else 0
        g.len[a] = float(length[a]) if (length is not None and a < dim) else 1.0
    return g


def _bc_array(bc):
    arr = (ctypes.c_int * 6)()
    for k, v in enumerate(bc):
        arr[k] = int(v)
    return arr


def _dev(x, name):
    """float64 contiguous CUDA tensor (from numpy or torch)."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name}: expected numpy array or torch tensor")
    x = x.to(device="cuda", dtype=torch.float64).contiguous()
    return x


def _host(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def plan(dim, n, rho, lam, mu, omega, bc, length=None, **opts):
    """Time-step plan on the host (no GPU): dict with nt, dt, c, lambda_bound."""
    g = make_grid(dim, n, length)
    r, l, m = _host(rho), _host(lam), _host(mu)
    o = default_opts(**opts)
    info = Info()
    st = lib.elwh_plan(ctypes.byref(g), r.ctypes.data, l.ctypes.data, m.ctypes.data, float(omega),
                       _bc_array(bc), ctypes.byref(o), ctypes.byref(info))
    if st != OK:
        raise ElwhError(st, lib.elwh_last_error(None).decode())
    return {"nt": info.nt, "dt": info.dt, "c": info.c, "lambda_bound": info.lambda_bound}


def dot_M_noalloc(dim, n, rho, bc, x, y, stream=None):
    """(x, y)_M without a context and without device allocation
    (elwh_dot_M_noalloc); rho, x, y CUDA float64 tensors in node layout."""
    g = make_grid(dim, n)
    for name, t in (("rho", rho), ("x", x), ("y", y)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError(f"{name}: expected a contiguous float64 CUDA tensor")
    s = (torch.cuda.current_stream() if stream is None else stream).cuda_stream
    r = ctypes.c_double()
    st = lib.elwh_dot_M_noalloc(ctypes.byref(g), rho.data_ptr(), _bc_array(bc), x.data_ptr(), y.data_ptr(),
                                ctypes.c_void_p(s), ctypes.byref(r))
    if st != OK:
        raise ElwhError(st, lib.elwh_last_error(None).decode())
    return r.value


def stream_triad(a, b, c, s=3.0, stream=None):
    """a = b + s c on the GPU (elwh_stream_triad), asynchronous; a, b, c
    contiguous float64 CUDA tensors of one length (a multiple of 4)."""
    n = a.numel()
    if not all(isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
               and t.numel() == n for t in (a, b, c)):
        raise TypeError("expected three contiguous float64 CUDA tensors of one length")
    st = (torch.cuda.current_stream() if stream is None else stream).cuda_stream
    r = lib.elwh_stream_triad(a.data_ptr(), b.data_ptr(), c.data_ptr(), float(s), int(n), ctypes.c_void_p(st))
    if r != OK:
        raise ElwhError(r, "elwh_stream_triad")


def filter_diagnostics(nt, periods=1, omega=1.0, scheme=0):
    """Discrete-filter accuracy of App. B (host only): dict with r_star, gap,
    beta_max, r_max, lambda_lo, lambda_hi (see elwh_filter_diagnostics)."""
    d = FilterDiag()
    st = lib.elwh_filter_diagnostics(int(nt), int(periods), float(omega), int(scheme), ctypes.byref(d))
    if st != OK:
        raise ElwhError(st, lib.elwh_last_error(None).decode())
    return {k: getattr(d, k) for k, _ in FilterDiag._fields_}


def plan_mapped(x, y, rho, lam, mu, omega, bc=(0, 0, 0, 0), **opts):
    """Time-step plan of a mapped 2-D grid on the host (no GPU); x, y, rho,
    lam, mu node arrays of shape (n_r + 1, n_q + 1); bc the sides
    (-q, +q, -r, +r)."""
    xs, ys = _host(x), _host(y)
    nr, nq = xs.shape[0] - 1, xs.shape[1] - 1
    g = make_grid(2, (nq, nr))
    r, l, m = _host(rho), _host(lam), _host(mu)
    o = default_opts(**opts)
    info = Info()
    st = lib.elwh_plan_mapped(ctypes.byref(g), xs.ctypes.data, ys.ctypes.data, r.ctypes.data, l.ctypes.data,
                              m.ctypes.data, float(omega), _bc_array(bc), ctypes.byref(o),
                              ctypes.byref(info))
    if st != OK:
        raise ElwhError(st, lib.elwh_last_error(None).decode())
    return {"nt": info.nt, "dt": info.dt, "c": info.c, "lambda_bound": info.lambda_bound}


class Context:
    """One El-WaveHoltz problem on the GPU (wraps elwh_create / elwh_destroy)."""

    def __init__(self, dim, n, rho, lam, mu, omega, bc, length=None, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libelwh needs a GPU")
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.node_shape = tuple(self.n[a] + 1 for a in reversed(range(dim)))
        self.field_shape = (dim,) + self.node_shape
        self.stream = torch.cuda.current_stream() if stream is None else stream
        g = make_grid(dim, n, length)
        o = default_opts(stream=self.stream.cuda_stream, **opts)
        self._r, self._l, self._m = _dev(rho, "rho"), _dev(lam, "lam"), _dev(mu, "mu")
        for t in (self._r, self._l, self._m):
            if tuple(t.shape) != self.node_shape:
                raise ValueError(f"material shape {tuple(t.shape)} != {self.node_shape}")
        h = ctypes.c_void_p()
        st = lib.elwh_create(ctypes.byref(g), self._r.data_ptr(), self._l.data_ptr(), self._m.data_ptr(),
                             float(omega), _bc_array(bc), ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise ElwhError(st, lib.elwh_last_error(None).decode())
        self._h = h
        self.opts = o
        del self._r, self._l, self._m          # the library copied them

    def close(self):
        if getattr(self, "_h", None):
            lib.elwh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise ElwhError(st, lib.elwh_last_error(self._h).decode())

    def _field(self, x, name):
        t = _dev(x, name)
        if tuple(t.shape) != self.field_shape:
            raise ValueError(f"{name} shape {tuple(t.shape)} != {self.field_shape}")
        return t

    def info(self):
        i = Info()
        self._check(lib.elwh_query(self._h, ctypes.byref(i)))
        return i.as_dict()

    def apply_filter(self, u0, f=None, out=None):
        u0 = self._field(u0, "u0")
        ft = self._field(f, "f") if f is not None else None
        out = torch.empty(self.field_shape, dtype=torch.float64, device="cuda") if out is None else out
        self._check(lib.elwh_apply_filter(self._h, u0.data_ptr(), ft.data_ptr() if ft is not None else None,
                                          out.data_ptr()))
        return out

    def apply_A(self, x, out=None):
        x = self._field(x, "x")
        out = torch.empty(self.field_shape, dtype=torch.float64, device="cuda") if out is None else out
        self._check(lib.elwh_apply_A(self._h, x.data_ptr(), out.data_ptr()))
        return out

    def dot_M(self, x, y):
        x, y = self._field(x, "x"), self._field(y, "y")
        r = ctypes.c_double()
        self._check(lib.elwh_dot_M(self._h, x.data_ptr(), y.data_ptr(), ctypes.byref(r)))
        return r.value

    def solve(self, f, x0=None, tol=1e-10, maxit=1000, raise_on_fail=True):
        f = self._field(f, "f")
        x0t = self._field(x0, "x0") if x0 is not None else None
        v = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        info = Info()
        st = lib.elwh_solve(self._h, f.data_ptr(), x0t.data_ptr() if x0t is not None else None, float(tol),
                            int(maxit), v.data_ptr(), ctypes.byref(info))
        d = info.as_dict()
        d["status"] = STATUS_NAMES[st]
        if st != OK and raise_on_fail:
            self._check(st)
        return v, d

    # two-field operator (impedance faces)
    def apply_filter2(self, u0, u1, f=None):
        """(out0, out1) = Pi_h [u0; u1]: filtered displacement and velocity."""
        u0, u1 = self._field(u0, "u0"), self._field(u1, "u1")
        ft = self._field(f, "f") if f is not None else None
        o0 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        o1 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        self._check(lib.elwh_apply_filter2(self._h, u0.data_ptr(), u1.data_ptr(),
                                           ft.data_ptr() if ft is not None else None, o0.data_ptr(), o1.data_ptr()))
        return o0, o1

    def apply_A2(self, x0, x1):
        x0, x1 = self._field(x0, "x0"), self._field(x1, "x1")
        y0 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        y1 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        self._check(lib.elwh_apply_A2(self._h, x0.data_ptr(), x1.data_ptr(), y0.data_ptr(), y1.data_ptr()))
        return y0, y1

    def solve2(self, f, x0=None, x1=None, tol=1e-10, maxit=1000, raise_on_fail=True):
        """GMRES for the two-field fixed point: (u0, u1, info)."""
        f = self._field(f, "f")
        a = self._field(x0, "x0") if x0 is not None else None
        b = self._field(x1, "x1") if x1 is not None else None
        v0 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        v1 = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        info = Info()
        st = lib.elwh_solve2(self._h, f.data_ptr(), a.data_ptr() if a is not None else None,
                             b.data_ptr() if b is not None else None, float(tol), int(maxit), v0.data_ptr(),
                             v1.data_ptr(), ctypes.byref(info))
        d = info.as_dict()
        d["status"] = STATUS_NAMES[st]
        if st != OK and raise_on_fail:
            self._check(st)
        return v0, v1, d

    # stepwise CG
    def cg_begin(self, f, x0=None):
        f = self._field(f, "f")
        x0t = self._field(x0, "x0") if x0 is not None else None
        self._check(lib.elwh_cg_begin(self._h, f.data_ptr(), x0t.data_ptr() if x0t is not None else None))

    def cg_iterate(self, k, tol=0.0):
        r = ctypes.c_double()
        self._check(lib.elwh_cg_iterate(self._h, int(k), float(tol), ctypes.byref(r)))
        return r.value

    def set_tile(self, prec, vec, rows):
        self._check(lib.elwh_set_tile(self._h, int(prec), int(vec), int(rows)))

    def get_tile(self, prec):
        v, r = ctypes.c_int(), ctypes.c_int()
        self._check(lib.elwh_get_tile(self._h, int(prec), ctypes.byref(v), ctypes.byref(r)))
        return v.value, r.value

    def autotune(self, prec, reps=2):
        us = ctypes.c_double()
        self._check(lib.elwh_autotune(self._h, int(prec), int(reps), ctypes.byref(us)))
        return us.value

    def profile_enable(self, on=True):
        self._check(lib.elwh_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """Summed fused-step kernel time (ms) and launch counts since the last read."""
        ts, ti = ctypes.c_double(), ctypes.c_double()
        ns, ni = ctypes.c_int(), ctypes.c_int()
        self._check(lib.elwh_profile_read(self._h, ctypes.byref(ts), ctypes.byref(ns), ctypes.byref(ti),
                                          ctypes.byref(ni)))
        return {"step_ms": ts.value, "nstep": ns.value, "init_ms": ti.value, "ninit": ni.value}

    def cg_result(self):
        v = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
        info = Info()
        self._check(lib.elwh_cg_result(self._h, v.data_ptr(), ctypes.byref(info)))
        return v, info.as_dict()


class MappedContext(Context):
    """One problem on a mapped 2-D grid (wraps elwh_create_mapped): x, y are
    the node coordinates, shape (n_r + 1, n_q + 1), q along the last axis;
    bc = (-q, +q, -r, +r) sides, q sides Dirichlet, r sides Dirichlet (0) or
    traction-free (1).  Every Context method applies."""

    def __init__(self, x, y, rho, lam, mu, omega, bc=(0, 0, 0, 0), stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libelwh needs a GPU")
        xs = _dev(x, "x")
        ys = _dev(y, "y")
        if xs.dim() != 2 or tuple(ys.shape) != tuple(xs.shape):
            raise ValueError("x and y must be node arrays of one 2-D shape")
        nr, nq = xs.shape[0] - 1, xs.shape[1] - 1
        self.dim = 2
        self.n = (nq, nr)
        self.node_shape = (nr + 1, nq + 1)
        self.field_shape = (2,) + self.node_shape
        self.stream = torch.cuda.current_stream() if stream is None else stream
        g = make_grid(2, (nq, nr))
        o = default_opts(stream=self.stream.cuda_stream, **opts)
        r, l, m = _dev(rho, "rho"), _dev(lam, "lam"), _dev(mu, "mu")
        for t in (r, l, m):
            if tuple(t.shape) != self.node_shape:
                raise ValueError(f"material shape {tuple(t.shape)} != {self.node_shape}")
        h = ctypes.c_void_p()
        st = lib.elwh_create_mapped(ctypes.byref(g), xs.data_ptr(), ys.data_ptr(), r.data_ptr(), l.data_ptr(),
                                    m.data_ptr(), float(omega), _bc_array(bc), ctypes.byref(o),
                                    ctypes.byref(h))
        if st != OK:
            raise ElwhError(st, lib.elwh_last_error(None).decode())
        self._h = h
        self.opts = o


class MappedContext3(Context):
    """One problem on a mapped 3-D grid (wraps elwh_create_mapped3): x, y, z
    are the node coordinates, shape (n_s + 1, n_r + 1, n_q + 1), q along the
    last axis; bc = (-q, +q, -r, +r, -s, +s) faces, q and r faces Dirichlet,
    s faces Dirichlet (0) or traction-free (1).  Every Context method applies."""

    def __init__(self, x, y, z, rho, lam, mu, omega, bc=(0,) * 6, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libelwh needs a GPU")
        xs, ys, zs = _dev(x, "x"), _dev(y, "y"), _dev(z, "z")
        if xs.dim() != 3 or tuple(ys.shape) != tuple(xs.shape) or tuple(zs.shape) != tuple(xs.shape):
            raise ValueError("x, y and z must be node arrays of one 3-D shape")
        ns, nr, nq = (k - 1 for k in xs.shape)
        self.dim = 3
        self.n = (nq, nr, ns)
        self.node_shape = tuple(xs.shape)
        self.field_shape = (3,) + self.node_shape
        self.stream = torch.cuda.current_stream() if stream is None else stream
        g = make_grid(3, (nq, nr, ns))
        o = default_opts(stream=self.stream.cuda_stream, **opts)
        r, l, m = _dev(rho, "rho"), _dev(lam, "lam"), _dev(mu, "mu")
        for t in (r, l, m):
            if tuple(t.shape) != self.node_shape:
                raise ValueError(f"material shape {tuple(t.shape)} != {self.node_shape}")
        h = ctypes.c_void_p()
        st = lib.elwh_create_mapped3(ctypes.byref(g), xs.data_ptr(), ys.data_ptr(), zs.data_ptr(), r.data_ptr(),
                                     l.data_ptr(), m.data_ptr(), float(omega), _bc_array(bc), ctypes.byref(o),
                                     ctypes.byref(h))
        if st != OK:
            raise ElwhError(st, lib.elwh_last_error(None).decode())
        self._h = h
        self.opts = o


def plan_mapped3(x, y, z, rho, lam, mu, omega, bc=(0,) * 6, **opts):
    """Time-step plan of a mapped 3-D grid on the host (no GPU)."""
    xs, ys, zs = _host(x), _host(y), _host(z)
    ns, nr, nq = (k - 1 for k in xs.shape)
    g = make_grid(3, (nq, nr, ns))
    r, l, m = _host(rho), _host(lam), _host(mu)
    o = default_opts(**opts)
    info = Info()
    st = lib.elwh_plan_mapped3(ctypes.byref(g), xs.ctypes.data, ys.ctypes.data, zs.ctypes.data, r.ctypes.data,
                               l.ctypes.data, m.ctypes.data, float(omega), _bc_array(bc), ctypes.byref(o),
                               ctypes.byref(info))
    if st != OK:
        raise ElwhError(st, lib.elwh_last_error(None).decode())
    return {"nt": info.nt, "dt": info.dt, "c": info.c, "lambda_bound": info.lambda_bound}


def context_from_case(case, **opts):
    """Context for an inputs.Case."""
    return Context(case.dim, case.n, case.rho, case.lam, case.mu, case.omega, case.bc, length=case.length, **opts)


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = t.data_ptr() if t is not None else None
    return arr


class Batch:
    """A ragged batch of 2-D problems solved together (elwh_batch_*)."""

    def __init__(self, cases, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libelwh needs a GPU")
        self.cases = list(cases)
        n = len(self.cases)
        grids = (Grid * n)()
        bc = (ctypes.c_int * (6 * n))()
        om = (ctypes.c_double * n)()
        keep = []
        for k, c in enumerate(self.cases):
            if c.dim != 2:
                raise ValueError("batches hold 2-D problems")
            g = make_grid(2, c.n, c.length)
            grids[k] = g
            for q in range(6):
                bc[6 * k + q] = int(c.bc[q]) if q < 4 else 0
            om[k] = float(c.omega)
            keep.append((_dev(c.rho, "rho"), _dev(c.lam, "lam"), _dev(c.mu, "mu")))
        self.field_shapes = [(2,) + c.node_shape for c in self.cases]
        self.stream = torch.cuda.current_stream() if stream is None else stream
        o = default_opts(stream=self.stream.cuda_stream, **opts)
        h = ctypes.c_void_p()
        st = lib.elwh_batch_create(n, grids, _ptr_array([k[0] for k in keep]), _ptr_array([k[1] for k in keep]),
                                   _ptr_array([k[2] for k in keep]), om, bc, ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise ElwhError(st, lib.elwh_batch_last_error(None).decode())
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            lib.elwh_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on):
        lib.elwh_batch_set_graph(self._h, 1 if on else 0)

    def solve(self, fs, x0s=None, tol=1e-8, maxit=1000, raise_on_fail=False):
        ft = [_dev(f, "f") for f in fs]
        xt = [(_dev(x, "x0") if x is not None else None) for x in (x0s or [None] * self.n)]
        vs = [torch.empty(s, dtype=torch.float64, device="cuda") for s in self.field_shapes]
        infos = (Info * self.n)()
        st = lib.elwh_batch_solve(self._h, _ptr_array(ft), _ptr_array(xt) if x0s is not None else None, float(tol),
                                  int(maxit), _ptr_array(vs), infos)
        if st != OK and raise_on_fail:
            raise ElwhError(st, lib.elwh_batch_last_error(self._h).decode())
        return vs, [infos[k].as_dict() for k in range(self.n)], STATUS_NAMES[st]

    def stats(self):
        sec = ctypes.c_double()
        ticks = ctypes.c_longlong()
        t64 = (ctypes.c_int * 2)()
        t32 = (ctypes.c_int * 2)()
        lib.elwh_batch_stats(self._h, ctypes.byref(sec), ctypes.byref(ticks), t64, t32)
        return {"seconds": sec.value, "ticks": ticks.value, "tile64": list(t64), "tile32": list(t32)}


class WarmStartNet:
    """The warm-start network of the library (elwh_ws_*).  Tensors are torch
    float32 CUDA tensors in NHWC layout."""

    def __init__(self, max_batch, H, W=None, seed=0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libelwh needs a GPU")
        W = H if W is None else W
        self.H, self.W, self.max_batch = H, W, max_batch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        st = lib.elwh_ws_create(int(max_batch), int(H), int(W), int(seed), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h))
        if st != OK:
            raise ElwhError(st, lib.elwh_ws_last_error(None).decode())
        self._h = h
        self.nparam = lib.elwh_ws_num_params(h)

    def close(self):
        if getattr(self, "_h", None):
            lib.elwh_ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise ElwhError(st, lib.elwh_ws_last_error(self._h).decode())

    def get_params(self):
        out = np.empty(self.nparam, dtype=np.float32)
        k = ctypes.c_double()
        self._check(lib.elwh_ws_params(self._h, out.ctypes.data, None, ctypes.byref(k), None))
        return out, k.value

    def set_params(self, theta=None, out_scale=None):
        t = None if theta is None else np.ascontiguousarray(theta, dtype=np.float32)
        k = None if out_scale is None else ctypes.byref(ctypes.c_double(float(out_scale)))
        self._check(lib.elwh_ws_params(self._h, None, t.ctypes.data if t is not None else None, None, k))

    def forward(self, x):
        B = x.shape[0]
        y = torch.empty((B, self.H, self.W, 2), dtype=torch.float32, device="cuda")
        self._check(lib.elwh_ws_forward(self._h, B, x.data_ptr(), y.data_ptr()))
        return y

    def loss_grad(self, x, y, w, want_grad=True):
        loss = ctypes.c_float()
        g = np.empty(self.nparam, dtype=np.float32) if want_grad else None
        self._check(lib.elwh_ws_loss_grad(self._h, x.shape[0], x.data_ptr(), y.data_ptr(), w.data_ptr(),
                                          ctypes.byref(loss), g.ctypes.data if g is not None else None))
        return loss.value, g

    def train_step(self, x, y, w, lr):
        loss = ctypes.c_float()
        self._check(lib.elwh_ws_train_step(self._h, x.shape[0], x.data_ptr(), y.data_ptr(), w.data_ptr(),
                                           float(lr), ctypes.byref(loss)))
        return loss.value

    def features(self, cases_dev, omega_dev, x_out, w_out):
        """cases_dev: list of (rho, lam, mu, f) CUDA float64 tensors."""
        B = len(cases_dev)
        n = self.H
        self._check(lib.elwh_ws_features(self._h, B, n, _ptr_array([c[0] for c in cases_dev]),
                                         _ptr_array([c[1] for c in cases_dev]), _ptr_array([c[2] for c in cases_dev]),
                                         _ptr_array([c[3] for c in cases_dev]), omega_dev.data_ptr(),
                                         x_out.data_ptr(), w_out.data_ptr()))

    def from_field(self, fs, vs, omega_dev, y_out):
        self._check(lib.elwh_ws_from_field(self._h, len(fs), self.H, _ptr_array(fs), _ptr_array(vs),
                                           omega_dev.data_ptr(), y_out.data_ptr()))

    def normalize(self, y, w):
        """y[b] /= its w-weighted RMS (elwh_ws_normalize), in place."""
        self._check(lib.elwh_ws_normalize(self._h, y.shape[0], y.data_ptr(), w.data_ptr()))

    def predict(self, x, fs, omega_dev, x0s):
        self._check(lib.elwh_ws_predict(self._h, len(fs), self.H, x.data_ptr(), _ptr_array(fs),
                                        omega_dev.data_ptr(), _ptr_array(x0s)))
