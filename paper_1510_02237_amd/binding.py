"""Python binding of libpararealhip (argument marshalling only).

Every computation runs in the HIP library; this module converts arguments
and calls the C ABI declared in include/libpararealhip.h.  States are
numpy float64 arrays of shape (..., 3, nz, nx) (host memory) or torch
float64 CUDA tensors of the same shape (device memory, passed by pointer).
PyTorch is used only to hold device memory.

If the shared library has not been built, load() raises instead of
falling back to anything else.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpararealhip.so")

PR_OK, PR_EINVAL, PR_ENOMEM, PR_EDEVICE, PR_EUNSTABLE = 0, -1, -2, -3, -4
PR_EAGAIN, PR_EBUSY, PR_EDIVERGED, PR_ENOTFOUND = -5, -6, -7, -8
PR_MEM_HOST, PR_MEM_DEVICE = 0, 1
PR_FORM_BATCHED, PR_FORM_PLAIN, PR_FORM_STAGEWISE = 0, 1, 2
FORMS = {"batched": PR_FORM_BATCHED, "plain": PR_FORM_PLAIN,
         "stagewise": PR_FORM_STAGEWISE}


class PRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpararealhip error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("Lx", ctypes.c_double), ("Lz", ctypes.c_double),
                ("T", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("nu_f", ctypes.c_double), ("nu_c", ctypes.c_double),
                ("n_sound", ctypes.c_int32), ("rank_tol", ctypes.c_double),
                ("form", ctypes.c_int32), ("skip_converged", ctypes.c_int32),
                ("tile_nt", ctypes.c_int32), ("tile_zc", ctypes.c_int32),
                ("windows", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("V", ctypes.c_double), ("stop_tol", ctypes.c_double),
                ("gamma", ctypes.c_double),
                ("fine_acoustic_order", ctypes.c_int32),
                ("coarse_order", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double),
                ("ms_coarse_init", ctypes.c_double),
                ("ms_fine", ctypes.c_double), ("ms_update", ctypes.c_double),
                ("ms_chain", ctypes.c_double),
                ("iterations", ctypes.c_int32),
                ("rank", ctypes.c_int32 * 64),
                ("fine_point_steps", ctypes.c_int64),
                ("residual", ctypes.c_double * 64),
                ("tile_nt", ctypes.c_int32), ("tile_zc", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32
_INT = ctypes.c_int
_SIGS = {
    "pr_opts_default": (None, [ctypes.POINTER(Opts)]),
    "pr_check_stability": (_INT, [ctypes.POINTER(Grid), _D, _D, _D, _D,
                                  ctypes.POINTER(Opts),
                                  ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "pr_footprint": (_INT, [ctypes.POINTER(Grid), _I, _I,
                            ctypes.POINTER(ctypes.c_size_t)]),
    "pr_create": (_INT, [ctypes.POINTER(Grid), _D, _D, _D, _D, _I,
                         ctypes.POINTER(_P)]),
    "pr_create_ex": (_INT, [ctypes.POINTER(Grid), _D, _D, _D, _D, _I,
                            ctypes.POINTER(Opts), _P, ctypes.POINTER(_P)]),
    "pr_destroy": (None, [_P]),
    "pr_set_form": (_INT, [_P, _I]),
    "pr_set_mfma": (_INT, [_P, _I]),
    "pr_fine_sweep": (_INT, [_P, _P, _P, _I, _INT]),
    "pr_coarse_step": (_INT, [_P, _P, _P, _INT, _INT]),
    "pr_krylov_update": (_INT, [_P, _P, _P, _I, ctypes.POINTER(_I), _INT]),
    "pr_krylov_reset": (_INT, [_P]),
    "pr_reserve_basis": (_INT, [_P, _I]),
    "pr_solve": (_INT, [_P, _P, _I, _P, _P, _INT]),
    "pr_solve_parareal": (_INT, [_P, _P, _I, _P, _P, _INT]),
    "pr_serial_fine": (_INT, [_P, _P, _I, _P, _INT]),
    "pr_get_stats": (_INT, [_P, ctypes.POINTER(Stats)]),
    "pr_server_create": (_INT, [_INT, ctypes.c_size_t, _I, ctypes.POINTER(_P)]),
    "pr_submit": (_INT, [_P, ctypes.POINTER(Grid), _D, _D, _D, _D, _I, _I, _P,
                         ctypes.POINTER(ctypes.c_uint64)]),
    "pr_submit_ex": (_INT, [_P, ctypes.POINTER(Grid), _D, _D, _D, _D, _I, _I,
                            ctypes.POINTER(Opts), _P,
                            ctypes.POINTER(ctypes.c_uint64)]),
    "pr_poll": (_INT, [_P, ctypes.c_uint64, _P, ctypes.POINTER(_D)]),
    "pr_cancel": (_INT, [_P, ctypes.c_uint64]),
    "pr_server_drain": (_INT, [_P]),
    "pr_server_destroy": (None, [_P]),
    "pr_strerror": (ctypes.c_char_p, [_INT]),
    "pr_last_error": (ctypes.c_char_p, [_P]),
    "pr_server_last_error": (ctypes.c_char_p, [_P]),
}


def load(path=LIB_PATH):
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with "
            "`python -m paper_1510_02237_amd.build` (hipcc, gfx950)")
    # torch ships its own HIP runtime under the same soname; load it first
    # so that this library binds to the same runtime instead of a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _err(code, ctx=None):
    lib = load()
    msg = lib.pr_last_error(ctx).decode() if ctx is not None or code else ""
    return PRError(code, msg or lib.pr_strerror(code).decode())


SCHEMES = {"split": 0, "rk3": 1}


def default_opts(**kw):
    o = Opts()
    load().pr_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "form" and isinstance(v, str):
            v = FORMS[v]
        if k == "scheme" and isinstance(v, str):
            v = SCHEMES[v]
        setattr(o, k, v)
    return o


def grid(nx, nz, T=1.0, Lx=1.0, Lz=1.0):
    return Grid(int(nx), int(nz), float(Lx), float(Lz), float(T))


def check_stability(nx, nz, c_s, U, dt_f, dt_g, **opts):
    rf, rg = _D(), _D()
    rc = load().pr_check_stability(ctypes.byref(grid(nx, nz)), c_s, U, dt_f,
                                   dt_g, ctypes.byref(default_opts(**opts)),
                                   ctypes.byref(rf), ctypes.byref(rg))
    if rc:
        raise _err(rc)
    return rf.value, rg.value


def footprint(nx, nz, P, K):
    b = ctypes.c_size_t()
    rc = load().pr_footprint(ctypes.byref(grid(nx, nz)), P, K, ctypes.byref(b))
    if rc:
        raise _err(rc)
    return b.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Arg:
    """A state argument: (pointer, mem kind, keep-alive object)."""

    def __init__(self, x, shape_tail, writable=False):
        if _is_torch(x):
            import torch
            if x.dtype != torch.float64 or not x.is_cuda:
                raise TypeError("device states must be float64 CUDA tensors")
            if not x.is_contiguous():
                raise ValueError("device states must be contiguous")
            if tuple(x.shape[-3:]) != shape_tail:
                raise ValueError(f"state shape {tuple(x.shape)} != (..., {shape_tail})")
            torch.cuda.current_stream(x.device).synchronize()
            self.ptr, self.mem, self.obj = x.data_ptr(), PR_MEM_DEVICE, x
        else:
            a = np.asarray(x)
            if a.dtype != np.float64 or not a.flags.c_contiguous or (
                    writable and not a.flags.writeable):
                if writable:
                    raise ValueError("output must be a writable C-contiguous float64 array")
                a = np.ascontiguousarray(a, dtype=np.float64)
            if tuple(a.shape[-3:]) != shape_tail:
                raise ValueError(f"state shape {a.shape} != (..., {shape_tail})")
            self.ptr, self.mem, self.obj = a.ctypes.data, PR_MEM_HOST, a


def _like(x, shape):
    if _is_torch(x):
        import torch
        return torch.empty(shape, dtype=torch.float64, device=x.device)
    return np.empty(shape, dtype=np.float64)


class Context:
    """One KSE-Parareal problem (pr_create_ex)."""

    def __init__(self, nx, nz, c_s, U, dt_f, dt_g, P, T=1.0, Lx=1.0, Lz=1.0,
                 **opts):
        self.lib = load()
        self.nx, self.nz, self.P = int(nx), int(nz), int(P)
        self.shape = (3, self.nz, self.nx)
        self._h = _P()
        self.opts = default_opts(**opts)
        rc = self.lib.pr_create_ex(ctypes.byref(grid(nx, nz, T, Lx, Lz)),
                                   float(c_s), float(U), float(dt_f),
                                   float(dt_g), int(P),
                                   ctypes.byref(self.opts), None,
                                   ctypes.byref(self._h))
        if rc:
            raise _err(rc)

    @classmethod
    def from_problem(cls, prob, **opts):
        """From a workload dict (paper_1510_02237_amd.workloads.problem)."""
        o = dict(nu_f=prob["nu_f"], nu_c=prob["nu_c"],
                 n_sound=prob["n_sound"], rank_tol=prob["rank_tol"],
                 windows=prob.get("windows", 1),
                 scheme=prob.get("scheme", "split"), V=prob.get("V", 0.0),
                 gamma=prob.get("gamma", 0.0),
                 fine_acoustic_order=prob.get("fine_acoustic_order", 4),
                 coarse_order=prob.get("coarse_order", 1))
        o.update(opts)
        return cls(prob["nx"], prob["nz"], prob["c_s"], prob["U"],
                   prob["dt_f"], prob["dt_g"], prob["P"], T=prob["T"], **o)

    def close(self):
        if self._h:
            self.lib.pr_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc:
            raise _err(rc, self._h)

    def set_form(self, form):
        self._chk(self.lib.pr_set_form(self._h, FORMS.get(form, form)))

    def set_mfma(self, on):
        self._chk(self.lib.pr_set_mfma(self._h, 1 if on else 0))

    def fine_sweep(self, Q, out=None):
        q = _Arg(Q, self.shape)
        ns = int(np.prod(q.obj.shape[:-3])) if q.obj.ndim > 3 else 1
        out = _like(Q, q.obj.shape) if out is None else out
        o = _Arg(out, self.shape, writable=True)
        if o.mem != q.mem:
            raise ValueError("Q and FQ must live in the same memory")
        self._chk(self.lib.pr_fine_sweep(self._h, q.ptr, o.ptr, ns, q.mem))
        return out

    def coarse_step(self, q, use_krylov=False, out=None):
        a = _Arg(q, self.shape)
        out = _like(q, self.shape) if out is None else out
        o = _Arg(out, self.shape, writable=True)
        self._chk(self.lib.pr_coarse_step(self._h, a.ptr, o.ptr,
                                          1 if use_krylov else 0, a.mem))
        return out

    def krylov_update(self, Q, FQ):
        a = _Arg(Q, self.shape)
        b = _Arg(FQ, self.shape)
        m = int(np.prod(a.obj.shape[:-3])) if a.obj.ndim > 3 else 1
        r = _I()
        self._chk(self.lib.pr_krylov_update(self._h, a.ptr, b.ptr, m,
                                            ctypes.byref(r), a.mem))
        return r.value

    def krylov_reset(self):
        self._chk(self.lib.pr_krylov_reset(self._h))

    def reserve_basis(self, n):
        self._chk(self.lib.pr_reserve_basis(self._h, int(n)))

    def solve(self, u0, K, slices=False, parareal=False, out=None):
        a = _Arg(u0, self.shape)
        out = _like(u0, self.shape) if out is None else out
        o = _Arg(out, self.shape, writable=True)
        sl = _like(u0, (self.P + 1,) + self.shape) if slices else None
        sp = _Arg(sl, self.shape, writable=True).ptr if slices else None
        fn = self.lib.pr_solve_parareal if parareal else self.lib.pr_solve
        self._chk(fn(self._h, a.ptr, int(K), o.ptr, sp, a.mem))
        return (out, sl) if slices else out

    def serial_fine(self, u0, nslices=None, out=None):
        a = _Arg(u0, self.shape)
        out = _like(u0, self.shape) if out is None else out
        o = _Arg(out, self.shape, writable=True)
        # default: every slice of every window, i.e. [0, T]
        ns = self.P * self.opts.windows if nslices is None else int(nslices)
        self._chk(self.lib.pr_serial_fine(self._h, a.ptr, ns, o.ptr, a.mem))
        return out

    def stats(self):
        s = Stats()
        self._chk(self.lib.pr_get_stats(self._h, ctypes.byref(s)))
        return dict(ms_total=s.ms_total, ms_coarse_init=s.ms_coarse_init,
                    ms_fine=s.ms_fine, ms_update=s.ms_update,
                    ms_chain=s.ms_chain, iterations=s.iterations,
                    rank=list(s.rank[:s.iterations]),
                    fine_point_steps=s.fine_point_steps,
                    residual=list(s.residual[:s.iterations]),
                    tile_nt=s.tile_nt, tile_zc=s.tile_zc)
