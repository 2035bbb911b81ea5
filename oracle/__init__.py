"""Sequential FP64 oracle for the Hubbard exact-diagonalisation hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1204_3425_amd``) and never imports it.

The arithmetic lives in ``hubbard_oracle.c`` (plain C, built with gcc -O2, one
thread); this module only marshals arguments, except ``Model.lowest_states``,
which hands the dense H built from that C code to numpy's symmetric
eigen-solver, ``Model.observables``, which sums psi^2 against the
configuration bits with numpy, and ``Model.propagate``, which builds
exp(-i H t) from that same eigen-solver.  Every function cites the part
of Siro & Harju (arXiv:1204.3425) it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hubbard_oracle.c")
_SO = os.path.join(_HERE, "_hubbard_oracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single thread, no vectorising flags)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


class _Result(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int), ("converged", ctypes.c_int), ("e0", ctypes.c_double),
                ("residual", ctypes.c_double), ("rayleigh", ctypes.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_SO)
            L.orc_basis.restype = _i64
            L.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int, _p, _i64]
            L.orc_position.restype = _i64
            L.orc_position.argtypes = [_p, _i64, ctypes.c_uint32]
            L.orc_model_new.restype = _p
            L.orc_model_new.argtypes = [ctypes.c_int, _p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double]
            L.orc_model_new_bonds.restype = _p
            L.orc_model_new_bonds.argtypes = [ctypes.c_int, _p, _p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double]
            L.orc_model_free.argtypes = [_p]
            L.orc_dim.restype = _i64
            L.orc_dim.argtypes = [_p, ctypes.c_int]
            L.orc_nnz.restype = _i64
            L.orc_nnz.argtypes = [_p, ctypes.c_int]
            L.orc_export.argtypes = [_p, ctypes.c_int, _p, _p, _p, _p]
            L.orc_apply.argtypes = [_p, _p, _p]
            L.orc_apply_rows.argtypes = [_p, _p, _p, _i64, _p]
            L.orc_diagonal.argtypes = [_p, _p]
            L.orc_splitmix64.restype = ctypes.c_uint64
            L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
            L.orc_start_raw.argtypes = [ctypes.c_uint64, _i64, _p]
            L.orc_tridiag_min.restype = ctypes.c_double
            L.orc_tridiag_min.argtypes = [_p, _p, ctypes.c_int]
            L.orc_tridiag_vec.argtypes = [_p, _p, ctypes.c_int, ctypes.c_double, _p]
            L.orc_lanczos.restype = ctypes.c_int
            L.orc_lanczos.argtypes = [_p, _p, ctypes.c_double, ctypes.c_int, _p, _p, _p, _p,
                                      ctypes.POINTER(_Result)]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------ basis

def basis(ns: int, n: int) -> np.ndarray:
    """All ns-bit words with n bits set, ascending (Sec. 2.1, the ordering by
    the size of the binary number; bit i is site i)."""
    L = lib()
    count = L.orc_basis(ns, n, None, 0)
    out = np.zeros(count, dtype=np.uint32)
    L.orc_basis(ns, n, _ptr(out), count)
    return out


def position(states: np.ndarray, s: int) -> int:
    """Index of word s in the ascending list (i_sigma of eq. J-formula), -1 if absent."""
    states = np.ascontiguousarray(states, dtype=np.uint32)
    return int(lib().orc_position(_ptr(states), len(states), s))


def splitmix64(seed: int, k: int) -> int:
    """Output number k (k >= 1) of the SplitMix64 stream started at `seed`."""
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k))


def start_vector(seed: int, dim: int, normalise: bool = True) -> np.ndarray:
    """Random start vector of Alg. 1: f[J] = 2u - 1 from SplitMix64 counter J+1,
    scaled to unit norm in FP64 (Sec. 2.2)."""
    f = np.empty(dim, dtype=np.float64)
    lib().orc_start_raw(seed & (2**64 - 1), dim, _ptr(f))
    if normalise:
        f /= np.sqrt(np.dot(f, f))
    return f


def tridiag_min(a: np.ndarray, boff: np.ndarray) -> float:
    """Lowest eigenvalue of the tridiagonal T of eq. Tmatrix: diagonal a[0..m-1],
    off-diagonal boff[1..m-1] (boff[0] unused) by Sturm bisection."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    boff = np.ascontiguousarray(boff, dtype=np.float64)
    return float(lib().orc_tridiag_min(_ptr(a), _ptr(boff), len(a)))


def tridiag_vec(a: np.ndarray, boff: np.ndarray, lam: float) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    boff = np.ascontiguousarray(boff, dtype=np.float64)
    y = np.empty(len(a), dtype=np.float64)
    lib().orc_tridiag_vec(_ptr(a), _ptr(boff), len(a), lam, _ptr(y))
    return y


# ------------------------------------------------------------------ model

class Model:
    """The Hubbard Hamiltonian of eq. H restricted to one (N_up, N_dn) sector.

    edges: sequence of (i, j) site pairs, each bond listed once; the hermitian
    conjugate of every hop is implied by eq. H.
    """

    def __init__(self, ns, edges, n_up, n_dn, t=1.0, U=0.0):
        """t: one amplitude for every bond (eq. H), or a sequence with one
        amplitude per bond (the hop over bond k then has element -t[k] * sign)."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        self._edges = e
        self.ns, self.n_up, self.n_dn, self.U = ns, n_up, n_dn, float(U)
        if np.ndim(t) == 0:
            self.t = float(t)
            self._h = lib().orc_model_new(ns, _ptr(e), len(e), n_up, n_dn, self.t, self.U)
        else:
            amp = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
            assert amp.shape == (len(e),)
            self.t = amp.copy()
            self._h = lib().orc_model_new_bonds(ns, _ptr(e), _ptr(amp), len(e), n_up, n_dn, self.U)
        if not self._h:
            raise MemoryError("oracle model allocation failed")
        self.dim_up = int(lib().orc_dim(self._h, 0))
        self.dim_dn = int(lib().orc_dim(self._h, 1))
        self.dim = int(lib().orc_dim(self._h, 2))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_model_free(h)
            self._h = None

    def table(self, spin: int):
        """(states, row_start, col, val) of one spin's hopping matrix; rows sorted by column."""
        d = self.dim_up if spin == 0 else self.dim_dn
        nnz = int(lib().orc_nnz(self._h, spin))
        states = np.empty(d, dtype=np.uint32)
        rs = np.empty(d + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        val = np.empty(max(nnz, 1), dtype=np.float64)
        lib().orc_export(self._h, spin, _ptr(states), _ptr(rs), _ptr(col), _ptr(val))
        return states, rs, col[:nnz], val[:nnz]

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.dim,)
        y = np.empty_like(x)
        lib().orc_apply(self._h, _ptr(x), _ptr(y))
        return y

    def apply_rows(self, x: np.ndarray, rows) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.dim,)
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        assert rows.size == 0 or (rows.min() >= 0 and rows.max() < self.dim)
        y = np.empty(len(rows), dtype=np.float64)
        lib().orc_apply_rows(self._h, _ptr(x), _ptr(rows), len(rows), _ptr(y))
        return y

    def diagonal(self) -> np.ndarray:
        d = np.empty(self.dim, dtype=np.float64)
        lib().orc_diagonal(self._h, _ptr(d))
        return d

    def dense(self) -> np.ndarray:
        """H as a dense matrix, column by column through apply (small sectors only)."""
        assert self.dim <= 6000
        H = np.empty((self.dim, self.dim))
        e = np.zeros(self.dim)
        for c in range(self.dim):
            e[c] = 1.0
            H[:, c] = self.apply(e)
            e[c] = 0.0
        return H

    def lowest_states(self, k: int):
        """The k lowest eigenvalues of the sector Hamiltonian, repeated by
        multiplicity, and an orthonormal set of eigenvectors for them, one per
        row (Sec. 2.2 names the ground state and the lowest excited states as
        the wanted output of the method).  This is the definition written out:
        the full symmetric eigenproblem of the dense H (LAPACK through
        numpy.linalg.eigh), so small sectors only."""
        assert 1 <= k <= self.dim
        w, v = np.linalg.eigh(self.dense())
        return w[:k].copy(), np.ascontiguousarray(v[:, :k].T)

    def observables(self, psi: np.ndarray):
        """Site occupations of the state psi, <psi|O|psi> / <psi|psi> (Sec. 1:
        n_{i sigma} = c+_{i sigma} c_{i sigma}, which is diagonal in the basis of
        Sec. 2.1: bit i of the spin's configuration word).  Returns a dict:
          dens[s, i]     = <n_{i s}>,                  s = 0 up, 1 down
          corr[k, i, j]  = <n_{i a} n_{j b}>,          (a, b) = (up, up), (dn, dn), (up, dn) for k = 0, 1, 2
          docc           = <sum_i n_{i up} n_{i dn}>   (the operator of the interaction term of eq. H)
        Every term is the sum over J of psi_J^2 times the product of the bits,
        written with matrix products over the dim_up x dim_dn view of psi^2."""
        psi = np.asarray(psi, dtype=np.float64)
        assert psi.shape == (self.dim,)
        ns = self.ns
        su, _, _, _ = self.table(0)
        sd, _, _, _ = self.table(1)
        bu = ((su[:, None] >> np.arange(ns)) & 1).astype(np.float64)  # dim_up x ns
        bd = ((sd[:, None] >> np.arange(ns)) & 1).astype(np.float64)  # dim_dn x ns
        W = (psi * psi).reshape(self.dim_up, self.dim_dn)
        norm = W.sum()
        R = W.sum(axis=1)                       # weight of each up configuration
        Q = W.sum(axis=0)                       # weight of each down configuration
        dens = np.stack([bu.T @ R, bd.T @ Q]) / norm
        corr = np.stack([(bu * R[:, None]).T @ bu, (bd * Q[:, None]).T @ bd, bu.T @ W @ bd]) / norm
        return {"dens": dens, "corr": corr, "docc": float(np.trace(corr[2])), "norm2": float(norm)}

    def propagate(self, psi0: np.ndarray, t: float) -> np.ndarray:
        """exp(-i H t) psi0 for a complex psi0 (the time evolution that the
        product H.v also drives), written out as its definition: H = V diag(w) V^T
        from the dense symmetric eigenproblem (numpy.linalg.eigh), then
        V diag(exp(-i w t)) V^T psi0.  Small sectors only."""
        psi0 = np.asarray(psi0, dtype=np.complex128)
        assert psi0.shape == (self.dim,)
        w, V = np.linalg.eigh(self.dense())
        return V @ (np.exp(-1j * w * t) * (V.T @ psi0))

    def lanczos(self, f1: np.ndarray, tol: float = 1e-12, max_iter: int = 300, want_psi: bool = False):
        """Alg. 1 from the unit start vector f1; returns a dict with a_j, b_{j+1},
        the Ritz-value history, E0 and (optionally) psi, its residual and
        Rayleigh quotient."""
        f1 = np.ascontiguousarray(f1, dtype=np.float64)
        assert f1.shape == (self.dim,)
        a = np.zeros(max_iter)
        b = np.zeros(max_iter)
        eh = np.zeros(max_iter)
        psi = np.empty(self.dim) if want_psi else None
        res = _Result()
        rc = lib().orc_lanczos(self._h, _ptr(f1), tol, max_iter, _ptr(a), _ptr(b), _ptr(eh),
                               _ptr(psi) if psi is not None else None, ctypes.byref(res))
        if rc != 0:
            raise MemoryError("oracle Lanczos ran out of memory")
        m = res.n_iter
        out = {"a": a[:m].copy(), "b": b[:m].copy(), "e_hist": eh[:m].copy(), "n_iter": m,
               "converged": res.converged, "E0": res.e0}
        if want_psi:
            out.update(psi=psi, residual=res.residual, rayleigh=res.rayleigh)
        return out
