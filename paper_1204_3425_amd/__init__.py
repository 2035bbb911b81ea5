"""MI355X-native exact diagonalisation of the Hubbard model.

Python binding of the C ABI declared in ``include/hubbard.h``: the functions
here carry the same names as the C entry points and only marshal arguments
(torch CUDA tensors or raw device pointers in, host results out).  Every step
of the computation runs in the HIP library ``_hubbard.so`` built for gfx950;
there is no CPU fallback, and importing the package fails loudly when the
library has not been built (``python -m paper_1204_3425_amd.build``).

Method: Siro & Harju, "Exact diagonalization of the Hubbard model on graphics
processing units" (arXiv:1204.3425): basis and J order (Sec. 2.1), Lanczos
(Sec. 2.2, Alg. 1), Kronecker-split ELL hopping tables and the fused H.v
kernel (Sec. 4.2-4.3).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_hubbard.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "hubbard.h")

HUBBARD_OK = 0
HUBBARD_ENOCONV = 1
HUBBARD_EINVAL = -1
HUBBARD_ERANGE = -2
HUBBARD_ENOMEM = -3
HUBBARD_EDEVICE = -4
HUBBARD_EBUSY = -5
HUBBARD_FP64 = 0
HUBBARD_MIXED = 1
HUBBARD_SPIN_UP = 0
HUBBARD_SPIN_DN = 1
STOP_NAMES = {0: "max_iter", 1: "converged", 2: "breakdown", 3: "exhausted"}
DEFAULT_SEED = 12043425


class HubbardError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed with %d (%s): %s" % (where, code, _strerror(code), msg))
        self.code = code


class hubbard_info_t(ctypes.Structure):
    _fields_ = [("sites", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("n_edges", ctypes.c_int32), ("t", ctypes.c_double), ("U", ctypes.c_double),
                ("dim_up", ctypes.c_int64), ("dim_dn", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("w_up", ctypes.c_int32), ("w_dn", ctypes.c_int32), ("nnz_up", ctypes.c_int64),
                ("nnz_dn", ctypes.c_int64), ("device_bytes", ctypes.c_size_t), ("vector_bytes", ctypes.c_size_t),
                ("ld_pref", ctypes.c_int64)]


class hubbard_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("start", ctypes.c_void_p), ("psi", ctypes.c_void_p),
                ("a_out", ctypes.c_void_p), ("b_out", ctypes.c_void_p), ("e_out", ctypes.c_void_p)]


class hubbard_result(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("residual", ctypes.c_double), ("rayleigh", ctypes.c_double),
                ("err_est", ctypes.c_double), ("seconds", ctypes.c_double), ("seconds_per_iter", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("stop", ctypes.c_int32), ("status", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("psi_resident", ctypes.c_int32)]


class hubbard_prop_result(ctypes.Structure):
    _fields_ = [("err_est", ctypes.c_double), ("norm", ctypes.c_double), ("seconds", ctypes.c_double),
                ("n_steps", ctypes.c_int32), ("krylov_dim_max", ctypes.c_int32)]


class hubbard_request(ctypes.Structure):
    _fields_ = [("sites", ctypes.c_int32), ("edges", ctypes.c_void_p), ("n_edges", ctypes.c_int32),
                ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32), ("t", ctypes.c_double), ("U", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class hubbard_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double), ("result", hubbard_result)]


class hubbard_server_stats_t(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_uint64), ("reserved", ctypes.c_uint64), ("peak_reserved", ctypes.c_uint64),
                ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("pending", ctypes.c_uint64), ("max_active_batch", ctypes.c_int32),
                ("slots_used", ctypes.c_int32), ("solo_runs", ctypes.c_uint64)]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64.so.7, and
    # loading it first makes this library bind to that same instance (the
    # loader matches our libamdhip64.so.7 dependency to its soname) instead of
    # a second runtime from /opt/rocm, which would leave torch without a device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("the HIP library %s is not built; run `python -m paper_1204_3425_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "hubbard_build": [i32, vp, i32, i32, i32, dbl, dbl, ctypes.POINTER(vp)],
        "hubbard_build_bonds": [i32, vp, vp, i32, i32, i32, dbl, ctypes.POINTER(vp)],
        "hubbard_free": [vp],
        "hubbard_set_stream": [vp, vp],
        "hubbard_set_precision": [vp, i32],
        "hubbard_set_seed": [vp, u64],
        "hubbard_set_basis_limit": [vp, ctypes.c_size_t],
        "hubbard_apply": [vp, vp, vp],
        "hubbard_apply_ld": [vp, vp, i64, vp, i64],
        "hubbard_lanczos": [vp, dbl, i32, ctypes.POINTER(dbl), vp],
        "hubbard_lanczos_ex": [vp, ctypes.POINTER(hubbard_opts), ctypes.POINTER(hubbard_result)],
        "hubbard_info": [vp, ctypes.POINTER(hubbard_info_t)],
        "hubbard_export_basis": [vp, i32, vp],
        "hubbard_export_table": [vp, i32, vp, vp],
        "hubbard_start_raw": [u64, i64, vp, vp],
        "hubbard_lanczos_batch": [vp, i32, ctypes.POINTER(hubbard_opts), ctypes.POINTER(hubbard_result)],
        "hubbard_lowest_states": [vp, i32, ctypes.POINTER(hubbard_opts), vp, vp, ctypes.POINTER(hubbard_result)],
        "hubbard_observables": [vp, vp, vp, vp, vp],
        "hubbard_observables_noalloc": [vp, vp, vp, vp, vp],
        "hubbard_propagate": [vp, vp, vp, dbl, i32, i32, vp, ctypes.POINTER(hubbard_prop_result)],
        "hubbard_server_create": [ctypes.c_size_t, i32, ctypes.POINTER(vp)],
        "hubbard_server_submit": [vp, ctypes.POINTER(hubbard_request), ctypes.POINTER(ctypes.c_uint64)],
        "hubbard_server_poll": [vp, ctypes.POINTER(hubbard_completion), i32, ctypes.POINTER(ctypes.c_int), i32],
        "hubbard_server_stats": [vp, ctypes.POINTER(hubbard_server_stats_t)],
        "hubbard_server_destroy": [vp],
        "hubbard_admission_plan": [vp, i32, ctypes.c_uint64, ctypes.c_uint64, i32, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.hubbard_strerror.argtypes = [ctypes.c_int]
    L.hubbard_strerror.restype = ctypes.c_char_p
    L.hubbard_last_error.argtypes = []
    L.hubbard_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def _strerror(code):
    return _lib.hubbard_strerror(code).decode()


def hubbard_strerror(code: int) -> str:
    return _strerror(code)


def hubbard_last_error() -> str:
    return _lib.hubbard_last_error().decode()


def _check(rc, where, allow=(HUBBARD_OK,)):
    if rc not in allow:
        raise HubbardError(rc, where, hubbard_last_error())
    return rc


def _dev_ptr(t, dtype_name=None, numel=None, what="tensor"):
    """Device address of a torch CUDA tensor (checked) or a raw integer pointer."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor or a device pointer" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if dtype_name is not None and str(t.dtype) != "torch." + dtype_name:
        raise TypeError("%s must be %s, got %s" % (what, dtype_name, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (what, numel, t.numel()))
    return t.data_ptr()


def _current_stream():
    import torch
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        return torch.cuda.current_stream().cuda_stream
    return None


class Handle:
    """Owns one C handle; freed with hubbard_free when garbage-collected."""

    def __init__(self, ptr, sites, edges, n_up, n_dn, t, U):
        self.ptr = ptr
        self.sites, self.edges, self.n_up, self.n_dn, self.t, self.U = sites, edges, n_up, n_dn, t, U
        info = hubbard_info(self)
        self.dim_up, self.dim_dn, self.dim = info["dim_up"], info["dim_dn"], info["dim"]
        self.precision = HUBBARD_FP64

    def __del__(self):
        p = getattr(self, "ptr", None)
        if p and _lib is not None:
            _lib.hubbard_free(p)
            self.ptr = None

    @property
    def _as_parameter_(self):
        if not self.ptr:
            raise ValueError("handle already freed")
        return ctypes.c_void_p(self.ptr)

    @property
    def vec_dtype(self):
        return "float64" if self.precision == HUBBARD_FP64 else "float32"


def hubbard_build(sites, edges, n_up, n_dn, t=1.0, U=0.0) -> Handle:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    out = ctypes.c_void_p()
    _check(_lib.hubbard_build(int(sites), e.ctypes.data_as(ctypes.c_void_p), len(e), int(n_up), int(n_dn),
                              float(t), float(U), ctypes.byref(out)), "hubbard_build")
    return Handle(out.value, sites, [tuple(x) for x in e.tolist()], n_up, n_dn, float(t), float(U))


def hubbard_build_bonds(sites, edges, t, n_up, n_dn, U=0.0) -> Handle:
    """As hubbard_build with one hopping amplitude per bond (t: sequence, one per edge)."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    a = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(-1))
    if len(a) != len(e):
        raise ValueError("one amplitude per edge expected")
    out = ctypes.c_void_p()
    _check(_lib.hubbard_build_bonds(int(sites), e.ctypes.data_as(ctypes.c_void_p),
                                    a.ctypes.data_as(ctypes.c_void_p), len(e), int(n_up), int(n_dn), float(U),
                                    ctypes.byref(out)), "hubbard_build_bonds")
    return Handle(out.value, sites, [tuple(x) for x in e.tolist()], n_up, n_dn, a.copy(), float(U))


def hubbard_free(h: Handle):
    if h.ptr:
        _check(_lib.hubbard_free(ctypes.c_void_p(h.ptr)), "hubbard_free")
        h.ptr = None


def hubbard_set_stream(h: Handle, stream=None):
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    _check(_lib.hubbard_set_stream(h, stream), "hubbard_set_stream")


def hubbard_set_precision(h: Handle, precision: int):
    _check(_lib.hubbard_set_precision(h, int(precision)), "hubbard_set_precision")
    h.precision = int(precision)


def hubbard_set_basis_limit(h: Handle, nbytes: int):
    _check(_lib.hubbard_set_basis_limit(h, int(nbytes)), "hubbard_set_basis_limit")


def hubbard_set_seed(h: Handle, seed: int):
    _check(_lib.hubbard_set_seed(h, int(seed) & (2**64 - 1)), "hubbard_set_seed")


def hubbard_apply(h: Handle, x, y, stream="current"):
    """y = H x on the device (asynchronous on torch's current stream by default)."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    xp = _dev_ptr(x, h.vec_dtype, h.dim, "x")
    yp = _dev_ptr(y, h.vec_dtype, h.dim, "y")
    _check(_lib.hubbard_apply(h, xp, yp), "hubbard_apply")


def hubbard_apply_ld(h: Handle, x, ldx: int, y, ldy: int, stream="current"):
    """y = H x with x, y stored as dim_up rows at strides ldx, ldy (elements)."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    nx = (h.dim_up - 1) * ldx + h.dim_dn
    ny = (h.dim_up - 1) * ldy + h.dim_dn
    xp = _dev_ptr(x, h.vec_dtype, None, "x")
    yp = _dev_ptr(y, h.vec_dtype, None, "y")
    for t, need, what in ((x, nx, "x"), (y, ny, "y")):
        if not isinstance(t, int) and t.numel() < need:
            raise ValueError("%s needs at least %d elements for this stride" % (what, need))
    _check(_lib.hubbard_apply_ld(h, xp, int(ldx), yp, int(ldy)), "hubbard_apply_ld")


def hubbard_lanczos(h: Handle, tol: float, max_iter: int, psi=None, stream="current"):
    """Returns (status, E0); psi (optional) is a device FP64 tensor of dim elements."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    e0 = ctypes.c_double()
    rc = _check(_lib.hubbard_lanczos(h, float(tol), int(max_iter), ctypes.byref(e0),
                                     _dev_ptr(psi, "float64", h.dim, "psi")),
                "hubbard_lanczos", allow=(HUBBARD_OK, HUBBARD_ENOCONV))
    return rc, e0.value


def _opts(h, tol, max_iter, precision, seed, start, psi, hist):
    o = hubbard_opts()
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.precision = int(h.precision if precision is None else precision)
    o.seed = int(DEFAULT_SEED if seed is None else seed) & (2**64 - 1)
    o.start = _dev_ptr(start, "float64", h.dim, "start")
    o.psi = _dev_ptr(psi, "float64", h.dim, "psi")
    if hist is not None:
        o.a_out = hist[0].ctypes.data
        o.b_out = hist[1].ctypes.data
        o.e_out = hist[2].ctypes.data
    return o


def _result_dict(r: hubbard_result, hist):
    m = r.n_iter
    out = {"E0": r.e0, "n_iter": m, "stop": STOP_NAMES.get(r.stop, r.stop), "status": r.status,
           "residual": r.residual, "rayleigh": r.rayleigh, "err_est": r.err_est, "seconds": r.seconds,
           "seconds_per_iter": r.seconds_per_iter, "precision": r.precision, "psi_resident": r.psi_resident}
    if hist is not None:
        out["a"], out["b"], out["e_hist"] = hist[0][:m].copy(), hist[1][:m].copy(), hist[2][:m].copy()
    return out


def hubbard_lanczos_ex(h: Handle, tol=1e-12, max_iter=300, precision=None, seed=None, start=None, psi=None,
                       history=True, stream="current"):
    """Full-option Lanczos; returns a dict with E0, a_j, b_{j+1}, the Ritz history,
    stop reason, and (when psi is given) the FP64 residual and Rayleigh quotient."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    hist = [np.zeros(max_iter), np.zeros(max_iter), np.zeros(max_iter)] if history else None
    o = _opts(h, tol, max_iter, precision, seed, start, psi, hist)
    r = hubbard_result()
    _check(_lib.hubbard_lanczos_ex(h, ctypes.byref(o), ctypes.byref(r)), "hubbard_lanczos_ex",
           allow=(HUBBARD_OK, HUBBARD_ENOCONV))
    return _result_dict(r, hist)


def hubbard_lanczos_batch(handles, tol=1e-12, max_iter=300, precision=None, seeds=None, psis=None,
                          history=False, stream="current"):
    n = len(handles)
    if stream == "current":
        s = _current_stream()
        for h in handles:
            hubbard_set_stream(h, s)
    hists = [[np.zeros(max_iter), np.zeros(max_iter), np.zeros(max_iter)] if history else None for _ in range(n)]
    opts = (hubbard_opts * n)()
    for i, h in enumerate(handles):
        opts[i] = _opts(h, tol, max_iter, precision, None if seeds is None else seeds[i], None,
                        None if psis is None else psis[i], hists[i])
    res = (hubbard_result * n)()
    arr = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    rc = _lib.hubbard_lanczos_batch(arr, n, opts, res)
    if rc < 0:
        raise HubbardError(rc, "hubbard_lanczos_batch", hubbard_last_error())
    return [_result_dict(res[i], hists[i]) for i in range(n)]


def hubbard_lowest_states(h: Handle, k: int, tol=1e-12, max_iter=300, precision=None, seed=None, start=None,
                          psi=None, stream="current"):
    """The k lowest eigenvalues (with multiplicity) and, when psi is given (a
    contiguous device FP64 tensor of k * dim elements, e.g. shape (k, dim)),
    their eigenvectors; returns (E, results) with E a numpy array of k values
    and results one dict per state as hubbard_lanczos_ex returns."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    o = _opts(h, tol, max_iter, precision, seed, start, None, None)
    E = np.zeros(max(int(k), 1))
    res = (hubbard_result * max(int(k), 1))()
    pp = _dev_ptr(psi, "float64", int(k) * h.dim, "psi") if psi is not None else None
    _check(_lib.hubbard_lowest_states(h, int(k), ctypes.byref(o), E.ctypes.data, pp, res),
           "hubbard_lowest_states", allow=(HUBBARD_OK, HUBBARD_ENOCONV))
    return E[:k].copy(), [_result_dict(res[i], None) for i in range(int(k))]


def hubbard_observables(h: Handle, psi, stream="current") -> dict:
    """Site occupations of the state psi (device FP64 tensor of dim elements):
    dens (2, sites), corr (3, sites, sites) for (up,up), (dn,dn), (up,dn), and
    the double occupancy D."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    n = h.sites
    dens = np.zeros(2 * n)
    corr = np.zeros(3 * n * n)
    d = ctypes.c_double()
    _check(_lib.hubbard_observables(h, _dev_ptr(psi, "float64", h.dim, "psi"), dens.ctypes.data, corr.ctypes.data,
                                    ctypes.byref(d)), "hubbard_observables")
    return {"dens": dens.reshape(2, n), "corr": corr.reshape(3, n, n), "docc": d.value}


def hubbard_observables_noalloc(h: Handle, psi, stream="current") -> dict:
    """hubbard_observables through the entry point that allocates no device
    memory (partial sums in the library's static per-device scratch)."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    n = h.sites
    dens = np.zeros(2 * n)
    corr = np.zeros(3 * n * n)
    d = ctypes.c_double()
    _check(_lib.hubbard_observables_noalloc(h, _dev_ptr(psi, "float64", h.dim, "psi"), dens.ctypes.data,
                                            corr.ctypes.data, ctypes.byref(d)), "hubbard_observables_noalloc")
    return {"dens": dens.reshape(2, n), "corr": corr.reshape(3, n, n), "docc": d.value}


def hubbard_propagate(h: Handle, psi_re, psi_im, t: float, n_steps: int = 1, krylov_dim: int = 20,
                      stream="current") -> dict:
    """psi <- exp(-i H t) psi in place (device FP64 tensors of dim elements for the
    real and imaginary parts); returns the energy at every step boundary and the
    result record as a dict."""
    if stream == "current":
        hubbard_set_stream(h, _current_stream())
    energy = np.zeros(max(int(n_steps), 0) + 1)
    r = hubbard_prop_result()
    _check(_lib.hubbard_propagate(h, _dev_ptr(psi_re, "float64", h.dim, "psi_re"),
                                  _dev_ptr(psi_im, "float64", h.dim, "psi_im"), float(t), int(n_steps),
                                  int(krylov_dim), energy.ctypes.data, ctypes.byref(r)), "hubbard_propagate")
    return {"energy": energy, "err_est": r.err_est, "norm": r.norm, "seconds": r.seconds, "n_steps": r.n_steps,
            "krylov_dim_max": r.krylov_dim_max}


def hubbard_info(h: Handle) -> dict:
    info = hubbard_info_t()
    _check(_lib.hubbard_info(h, ctypes.byref(info)), "hubbard_info")
    return {name: getattr(info, name) for name, _ in hubbard_info_t._fields_}


def hubbard_export_basis(h: Handle, spin: int) -> np.ndarray:
    d = h.dim_up if spin == HUBBARD_SPIN_UP else h.dim_dn
    out = np.zeros(d, dtype=np.uint32)
    _check(_lib.hubbard_export_basis(h, int(spin), out.ctypes.data), "hubbard_export_basis")
    return out


def hubbard_export_table(h: Handle, spin: int):
    """(col, sgn) as flat column-major arrays of w_sigma * dim_sigma entries (Fig. ELL)."""
    info = hubbard_info(h)
    d = info["dim_up"] if spin == HUBBARD_SPIN_UP else info["dim_dn"]
    w = info["w_up"] if spin == HUBBARD_SPIN_UP else info["w_dn"]
    col = np.zeros(max(w * d, 1), dtype=np.int32)
    sgn = np.zeros(max(w * d, 1), dtype=np.int8)
    _check(_lib.hubbard_export_table(h, int(spin), col.ctypes.data, sgn.ctypes.data), "hubbard_export_table")
    return col[: w * d], sgn[: w * d]


def hubbard_start_raw(seed: int, dim: int, f, stream="current"):
    s = _current_stream() if stream == "current" else stream
    _check(_lib.hubbard_start_raw(int(seed) & (2**64 - 1), int(dim), _dev_ptr(f, "float64", dim, "f"), s),
           "hubbard_start_raw")


# ------------------------------------------------------------------ serving

class Server:
    """Owns one continuous-batching server (hubbard_server_destroy on close)."""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.hubbard_server_destroy(self.ptr)
            self.ptr = None

    @property
    def _as_parameter_(self):
        if not self.ptr:
            raise ValueError("server already destroyed")
        return ctypes.c_void_p(self.ptr)


def hubbard_server_create(hbm_budget: int, max_slots: int) -> Server:
    out = ctypes.c_void_p()
    _check(_lib.hubbard_server_create(int(hbm_budget), int(max_slots), ctypes.byref(out)), "hubbard_server_create")
    return Server(out.value)


def hubbard_server_submit(srv: Server, sites, edges, n_up, n_dn, t=1.0, U=0.0, tol=1e-10, max_iter=300,
                          precision=HUBBARD_MIXED, seed=DEFAULT_SEED, tag=0) -> int:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    r = hubbard_request(int(sites), e.ctypes.data, len(e), int(n_up), int(n_dn), float(t), float(U), float(tol),
                        int(max_iter), int(precision), int(seed) & (2**64 - 1), int(tag) & (2**64 - 1))
    rid = ctypes.c_uint64()
    _check(_lib.hubbard_server_submit(srv, ctypes.byref(r), ctypes.byref(rid)), "hubbard_server_submit")
    return rid.value


def hubbard_server_poll(srv: Server, cap: int = 256, timeout_us: int = 0):
    buf = (hubbard_completion * cap)()
    n = ctypes.c_int()
    _check(_lib.hubbard_server_poll(srv, buf, cap, ctypes.byref(n), int(timeout_us)), "hubbard_server_poll")
    out = []
    for k in range(n.value):
        c = buf[k]
        d = _result_dict(c.result, None)
        # the completion's own status (a rejected request has an empty result)
        d.update({"id": c.id, "tag": c.tag, "status": c.status, "t_submit": c.t_submit, "t_admit": c.t_admit,
                  "t_start": c.t_start, "t_done": c.t_done})
        out.append(d)
    return out


def hubbard_server_stats(srv: Server) -> dict:
    st = hubbard_server_stats_t()
    _check(_lib.hubbard_server_stats(srv, ctypes.byref(st)), "hubbard_server_stats")
    return {name: getattr(st, name) for name, _ in hubbard_server_stats_t._fields_}


def hubbard_server_destroy(srv: Server):
    if srv.ptr:
        _check(_lib.hubbard_server_destroy(ctypes.c_void_p(srv.ptr)), "hubbard_server_destroy")
        srv.ptr = None


def hubbard_admission_plan(footprints, budget: int, used: int, free_slots: int):
    fp = np.ascontiguousarray(np.asarray(footprints, dtype=np.uint64))
    take = np.zeros(len(fp), dtype=np.int32)
    n = _lib.hubbard_admission_plan(fp.ctypes.data, len(fp), int(budget), int(used), int(free_slots),
                                    take.ctypes.data)
    if n < 0:
        raise HubbardError(n, "hubbard_admission_plan", "")
    return take.tolist()


def sector_dim(sites: int, n_up: int, n_dn: int) -> int:
    return math.comb(sites, n_up) * math.comb(sites, n_dn)


__all__ = [n for n in dir() if n.startswith("hubbard_") or n.startswith("HUBBARD_")] + [
    "Handle", "Server", "HubbardError", "sector_dim", "LIB_PATH", "HEADER_PATH"]
