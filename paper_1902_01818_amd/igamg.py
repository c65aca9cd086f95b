"""ctypes binding of libigamg (include/igamg.h).  Argument marshalling only:
every step of the solver runs in the library's HIP kernels.  PyTorch
supplies device memory (float64 CUDA tensors) and the current stream.

If the shared library is missing this module raises at import time; there
is no fallback implementation.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigamg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libigamg.so is not built (run paper_1902_01818_amd.build.build())")
_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENOCONV = 0, -1, -2, -3, -4, 1
SIPG, CONFORMING = 0, 1
SMOOTHERS = {"hybrid": 0, "scms": 1, "gs": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
OUTERS = {"pcg": 0, "mg": 1, "fcg": 2, "ir": 3}
MANUFACTURED_SINE = 0
APPLIES = {"auto": 0, "sumfact": 1, "rows": 2}


class Patches(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_patches", ctypes.c_int),
                ("corners", ctypes.POINTER(ctypes.c_double)),
                ("elems", ctypes.POINTER(ctypes.c_int32)),
                ("degrees", ctypes.POINTER(ctypes.c_int32))]


class Options(ctypes.Structure):
    _fields_ = [("discretization", ctypes.c_int), ("smoother", ctypes.c_int),
                ("mu", ctypes.c_int), ("nu", ctypes.c_int),
                ("damping_tau", ctypes.c_double), ("scaling_delta", ctypes.c_double),
                ("precision", ctypes.c_int), ("outer", ctypes.c_int),
                ("gs_tile", ctypes.c_int), ("coarse_min", ctypes.c_int),
                ("timing", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("operator_apply", ctypes.c_int), ("graphs", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double))]


_vp = ctypes.c_void_p
_lib.igamg_default_options.argtypes = [ctypes.POINTER(Options)]
_lib.igamg_footprint.argtypes = [ctypes.POINTER(Patches), ctypes.c_int, ctypes.POINTER(Options),
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
_lib.igamg_setup.argtypes = [ctypes.POINTER(Patches), ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(Options), _vp, ctypes.POINTER(_vp)]
_lib.igamg_num_dofs.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.igamg_num_levels.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
_lib.igamg_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]
_lib.igamg_vcycle.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]
_lib.igamg_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, ctypes.POINTER(SolveInfo), _vp]
_lib.igamg_load_manufactured.argtypes = [_vp, ctypes.c_int, _vp, _vp]
_lib.igamg_l2_error.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp]
_lib.igamg_l2_error_noalloc.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        _vp]
_lib.igamg_memory.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.igamg_kernel_stats.argtypes = [_vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                    ctypes.c_int]
_lib.igamg_kernel_model.argtypes = [_vp, ctypes.c_char_p, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.igamg_set_timing.argtypes = [_vp, ctypes.c_char_p]
_lib.igamg_destroy.argtypes = [_vp]
_lib.igamg_strerror.restype = ctypes.c_char_p
_lib.igamg_last_error.restype = ctypes.c_char_p

class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("memory_budget", ctypes.c_size_t),
                ("device", ctypes.c_int)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("true_rel_residual", ctypes.c_double),
                ("n_dofs", ctypes.c_int64), ("footprint", ctypes.c_size_t),
                ("fallback_allocations", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_ready", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib.igamg_problem_size.argtypes = [ctypes.POINTER(Patches), ctypes.c_int, ctypes.POINTER(Options),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]
_lib.igamg_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
_lib.igamg_server_submit.argtypes = [_vp, ctypes.POINTER(Patches), ctypes.c_int, ctypes.c_double,
                                     ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int64)]
_lib.igamg_server_wait.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(RequestInfo)]
_lib.igamg_server_status.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t)]
_lib.igamg_server_destroy.argtypes = [_vp]

EXPORTED = ["igamg_default_options", "igamg_footprint", "igamg_setup", "igamg_num_dofs",
            "igamg_num_levels", "igamg_apply", "igamg_vcycle", "igamg_solve",
            "igamg_load_manufactured", "igamg_l2_error", "igamg_l2_error_noalloc",
            "igamg_memory", "igamg_kernel_stats",
            "igamg_kernel_model", "igamg_set_timing", "igamg_destroy", "igamg_strerror",
            "igamg_last_error", "igamg_problem_size", "igamg_server_create", "igamg_server_submit",
            "igamg_server_wait", "igamg_server_status", "igamg_server_destroy"]


class IgamgError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.igamg_last_error().decode()
        super().__init__("%s failed: %s (%s)" % (where, _lib.igamg_strerror(code).decode(), msg))


def _check(code, where, allow_noconv=False):
    if code == OK or (allow_noconv and code == ENOCONV):
        return code
    raise IgamgError(code, where)


def _stream(stream):
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    return _vp(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _patches(corners, elems, degree=None):
    """The patch description; degree: an int (the same on every patch, passed
    separately) or one degree per patch.  Returns (struct, arrays to keep
    alive, the degree argument of the C call)."""
    corners = np.ascontiguousarray(corners, dtype=np.float64)
    elems = np.ascontiguousarray(elems, dtype=np.int32)
    K, nc, d = corners.shape
    assert nc == 2 ** d and elems.shape == (K, d)
    degs = None
    if degree is not None and np.ndim(degree) > 0:
        degs = np.ascontiguousarray(degree, dtype=np.int32)
        assert degs.shape == (K,)
        degree = int(degs.max())
    P = Patches(d, K, corners.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                elems.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                None if degs is None else degs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return P, (corners, elems, degs), degree


def make_options(conforming=False, smoother="hybrid", tau=0.25, delta=0.1, mu=1, nu=1,
                 precision="fp64", outer="pcg", gs_tile=0, coarse_min=0, timing=False, max_rhs=0,
                 operator_apply="auto", graphs=False):
    o = Options()
    _lib.igamg_default_options(ctypes.byref(o))
    o.discretization = CONFORMING if conforming else SIPG
    o.smoother = SMOOTHERS[smoother]
    o.mu, o.nu = mu, nu
    o.damping_tau, o.scaling_delta = tau, delta
    o.precision = PRECISIONS[precision]
    o.outer = OUTERS[outer]
    o.gs_tile, o.coarse_min = gs_tile, coarse_min
    o.timing = 1 if timing else 0
    o.max_rhs = max_rhs
    o.operator_apply = APPLIES[operator_apply]
    o.graphs = 1 if graphs else 0
    return o


def footprint(corners, elems, degree, nrhs=0, **opts):
    """Device bytes of a setup for a batch of nrhs right-hand sides (0 = the
    options' max_rhs)."""
    P, keep, degree = _patches(corners, elems, degree)
    o = make_options(**opts)
    b = ctypes.c_size_t()
    _check(_lib.igamg_footprint(ctypes.byref(P), degree, ctypes.byref(o), nrhs, ctypes.byref(b)),
           "igamg_footprint")
    return int(b.value)


def problem_size(corners, elems, degree, **opts):
    """(N, levels) of a problem, computed on the host."""
    P, keep, degree = _patches(corners, elems, degree)
    o = make_options(**opts)
    n, lv = ctypes.c_int64(), ctypes.c_int()
    _check(_lib.igamg_problem_size(ctypes.byref(P), degree, ctypes.byref(o), ctypes.byref(n),
                                   ctypes.byref(lv)), "igamg_problem_size")
    return int(n.value), int(lv.value)


class Server:
    """igamg_server_*: continuous batching of solve requests (host arrays in/out)."""

    def __init__(self, slots=4, memory_budget=8 << 30, device=0):
        cfg = ServerConfig(slots, memory_budget, device)
        h = _vp()
        _check(_lib.igamg_server_create(ctypes.byref(cfg), ctypes.byref(h)), "igamg_server_create")
        self._h = h
        self._n = {}

    def submit(self, corners, elems, degree, rhs, sigma=5.0, tol=1e-8, maxit=200, **opts):
        P, keep, degree = _patches(corners, elems, degree)
        o = make_options(**opts)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        rid = ctypes.c_int64()
        _check(_lib.igamg_server_submit(self._h, ctypes.byref(P), degree, sigma, ctypes.byref(o),
                                        rhs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        rhs.size, tol, maxit, ctypes.byref(rid)),
               "igamg_server_submit")
        self._n[rid.value] = rhs.size
        return int(rid.value)

    def wait(self, rid):
        n = self._n.pop(rid)
        u = np.empty(n)
        info = RequestInfo()
        code = _lib.igamg_server_wait(self._h, rid, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in RequestInfo._fields_}
        d["status"] = code
        return u, d

    def status(self):
        q, r, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        used, peak = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.igamg_server_status(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(c),
                                        ctypes.byref(used), ctypes.byref(peak)), "igamg_server_status")
        return dict(queued=q.value, running=r.value, completed=c.value, reserved=used.value,
                    peak_reserved=peak.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.igamg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(t, n):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= n
    return _vp(t.data_ptr())


class Solver:
    """One problem instance: igamg_setup ... igamg_destroy."""

    def __init__(self, corners, elems, degree, sigma=5.0, stream=None, **opts):
        """degree: an int, or one degree per patch."""
        P, keep, degree = _patches(corners, elems, degree)
        o = make_options(**opts)
        h = _vp()
        _check(_lib.igamg_setup(ctypes.byref(P), degree, sigma, ctypes.byref(o), _stream(stream),
                                ctypes.byref(h)), "igamg_setup")
        self._h = h
        n = ctypes.c_int64()
        _check(_lib.igamg_num_dofs(h, ctypes.byref(n)), "igamg_num_dofs")
        self.n_dofs = int(n.value)
        lv = ctypes.c_int()
        _check(_lib.igamg_num_levels(h, ctypes.byref(lv)), "igamg_num_levels")
        self.n_levels = int(lv.value)

    def _cols(self, t):
        return t.numel() // self.n_dofs

    def apply(self, x, y=None, stream=None):
        y = torch.empty_like(x) if y is None else y
        _check(_lib.igamg_apply(self._h, _dptr(x, self.n_dofs), _dptr(y, self.n_dofs), self._cols(x),
                                _stream(stream)), "igamg_apply")
        return y

    def vcycle(self, f, u, stream=None):
        _check(_lib.igamg_vcycle(self._h, _dptr(f, self.n_dofs), _dptr(u, self.n_dofs), self._cols(f),
                                 _stream(stream)), "igamg_vcycle")
        return u

    def solve(self, rhs, u=None, tol=1e-8, maxit=500, use_initial_guess=False, history=False,
              stream=None):
        ncol = self._cols(rhs)
        if u is None:
            u = torch.zeros_like(rhs)
            use_initial_guess = False
        infos = (SolveInfo * ncol)()
        hist = []
        for j in range(ncol):
            if history:
                h = np.zeros(maxit + 1)
                hist.append(h)
                infos[j].history = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        code = _lib.igamg_solve(self._h, _dptr(rhs, self.n_dofs), _dptr(u, self.n_dofs), ncol, tol,
                                maxit, 1 if use_initial_guess else 0, infos, _stream(stream))
        _check(code, "igamg_solve", allow_noconv=True)
        out = []
        for j in range(ncol):
            d = dict(iterations=infos[j].iterations, rel_residual=infos[j].rel_residual,
                     true_rel_residual=infos[j].true_rel_residual, seconds=infos[j].seconds,
                     converged=infos[j].rel_residual <= tol)
            if history:
                d["history"] = hist[j][:infos[j].iterations + 1].copy()
            out.append(d)
        return u, out

    def load_manufactured(self, which=MANUFACTURED_SINE, stream=None):
        f = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda")
        _check(_lib.igamg_load_manufactured(self._h, which, _dptr(f, self.n_dofs), _stream(stream)),
               "igamg_load_manufactured")
        return f

    def l2_error(self, u, which=MANUFACTURED_SINE, stream=None):
        """||u_h - prod sin(pi x)||_{L2} of a finest-level coefficient vector."""
        e = ctypes.c_double()
        _check(_lib.igamg_l2_error(self._h, _dptr(u, self.n_dofs), which, ctypes.byref(e),
                                   _stream(stream)), "igamg_l2_error")
        return e.value

    def l2_error_noalloc(self, u, which=MANUFACTURED_SINE, stream=None):
        """As l2_error, through the entry point that allocates no device
        memory (its scratch is a static device array shared by every call on
        the GPU)."""
        e = ctypes.c_double()
        _check(_lib.igamg_l2_error_noalloc(self._h, _dptr(u, self.n_dofs), which, ctypes.byref(e),
                                           _stream(stream)), "igamg_l2_error_noalloc")
        return e.value

    def memory(self):
        b = ctypes.c_size_t()
        _check(_lib.igamg_memory(self._h, ctypes.byref(b)), "igamg_memory")
        return int(b.value)

    def kernel_stats(self, reset=False):
        cap = 256
        names = ctypes.create_string_buffer(32 * cap)
        ms = (ctypes.c_double * cap)()
        launches = (ctypes.c_int64 * cap)()
        cnt = ctypes.c_int()
        _check(_lib.igamg_kernel_stats(self._h, cap, names, ms, launches, ctypes.byref(cnt),
                                       1 if reset else 0), "igamg_kernel_stats")
        out = {}
        for i in range(cnt.value):
            nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = dict(ms=ms[i], launches=int(launches[i]))
        return out

    def kernel_model(self, family, level=-1, nrhs=1):
        b, f = ctypes.c_double(), ctypes.c_double()
        _check(_lib.igamg_kernel_model(self._h, family.encode(), level, nrhs, ctypes.byref(b),
                                       ctypes.byref(f)), "igamg_kernel_model")
        return b.value, f.value

    def set_timing(self, filter):
        """None = off, "" = all families, else a "<family>/<level>" prefix."""
        _check(_lib.igamg_set_timing(self._h, None if filter is None else filter.encode()),
               "igamg_set_timing")

    def close(self):
        if getattr(self, "_h", None):
            _lib.igamg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup(corners, elems, degree, sigma=5.0, **opts):
    return Solver(corners, elems, degree, sigma, **opts)
