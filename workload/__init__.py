"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method: it only produces lattices (as
lists of bonds), sector choices, interaction strengths, request traces and
random vectors.  Both the GPU library and the oracle receive these as inputs.

Lattices follow the paper's workloads (Sec. 5): a one-dimensional ring with
periodic boundaries and a two-dimensional square lattice with periodic
boundaries.  Sites of an Lx x Ly lattice are numbered x + Lx*y; bonds join
(x, y) to (x+1 mod Lx, y) and to (x, y+1 mod Ly).  Each unordered bond appears
once (a wrap-around bond that would repeat an existing one, as on a width-2
lattice, is dropped).  For per-bond amplitudes the square lattice also comes
with next-nearest (diagonal) bonds and their own amplitude (the t-t' lattice).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 12043425


def _dedupe(pairs):
    seen, out = set(), []
    for i, j in pairs:
        if i == j:
            continue
        key = (min(i, j), max(i, j))
        if key not in seen:
            seen.add(key)
            out.append((i, j))
    return out


def ring(ns: int):
    """Bonds of a periodic ring of ns sites: (i, i+1 mod ns)."""
    return _dedupe([(i, (i + 1) % ns) for i in range(ns)])


def chain(ns: int):
    """Bonds of an open chain."""
    return [(i, i + 1) for i in range(ns - 1)]


def torus(lx: int, ly: int):
    """Bonds of an lx x ly square lattice with periodic boundaries."""
    pairs = []
    for y in range(ly):
        for x in range(lx):
            s = x + lx * y
            pairs.append((s, (x + 1) % lx + lx * y))
            pairs.append((s, x + lx * ((y + 1) % ly)))
    return _dedupe(pairs)


def torus_tprime(lx: int, ly: int, t1: float, t2: float):
    """Bonds and per-bond amplitudes of the lx x ly periodic lattice with
    nearest-neighbour hopping t1 and next-nearest (both diagonals) t2:
    (edges, amplitudes), each unordered bond once."""
    nn = torus(lx, ly)
    diag = []
    for y in range(ly):
        for x in range(lx):
            s = x + lx * y
            diag.append((s, (x + 1) % lx + lx * ((y + 1) % ly)))
            diag.append((s, (x + 1) % lx + lx * ((y - 1) % ly)))
    seen = {(min(i, j), max(i, j)) for i, j in nn}
    extra = []
    for i, j in diag:
        key = (min(i, j), max(i, j))
        if i != j and key not in seen:
            seen.add(key)
            extra.append((i, j))
    return nn + extra, [float(t1)] * len(nn) + [float(t2)] * len(extra)


@dataclasses.dataclass(frozen=True)
class Problem:
    name: str
    sites: int
    edges: tuple
    n_up: int
    n_dn: int
    t: float
    U: float
    seed: int

    @property
    def dim_up(self):
        return math.comb(self.sites, self.n_up)

    @property
    def dim_dn(self):
        return math.comb(self.sites, self.n_dn)

    @property
    def dim(self):
        return self.dim_up * self.dim_dn

    def edge_array(self) -> np.ndarray:
        return np.asarray(self.edges, dtype=np.int32).reshape(-1, 2)


def problem(name, sites, edges, n_up, n_dn, t=1.0, U=0.0, seed=BASE_SEED) -> Problem:
    return Problem(name, sites, tuple(tuple(e) for e in edges), n_up, n_dn, float(t), float(U), int(seed))


# The workloads of the benchmark configurations.
def ring8() -> Problem:
    """Ring, 8 sites, 4 up + 4 down, t=1, U=4 (dim 4,900)."""
    return problem("ring8_4u4d_U4", 8, ring(8), 4, 4, 1.0, 4.0)


def ring14() -> Problem:
    """Ring, 14 sites, 7 up + 7 down, t=1, U=4 (dim 11,778,624)."""
    return problem("ring14_7u7d_U4", 14, ring(14), 7, 7, 1.0, 4.0)


def square4x4() -> Problem:
    """4x4 periodic square lattice, 8 up + 8 down, t=1, U=8 (dim 165,636,900)."""
    return problem("square4x4_8u8d_U8", 16, torus(4, 4), 8, 8, 1.0, 8.0)


def batch64(count: int = 64, seed: int = BASE_SEED):
    """Independent small solves: rings of 10..12 sites, N_up and N_dn drawn
    uniformly from [floor(Ns/2)-2, floor(Ns/2)], U uniform in [0, 16], t=1,
    instance i seeded with seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        ns = int(rng.integers(10, 13))
        h = ns // 2
        nu = int(rng.integers(h - 2, h + 1))
        nd = int(rng.integers(h - 2, h + 1))
        U = float(rng.uniform(0.0, 16.0))
        out.append(problem("batch%02d_ring%d_%du%dd" % (i, ns, nu, nd), ns, ring(ns), nu, nd, 1.0, U, seed + i))
    return out


def serving_trace(count: int = 2000, rate_per_s: float = 50.0, seed: int = BASE_SEED):
    """Request stream: lattice family uniform over {3x4 torus, 4x4 torus, ring};
    tori take N_up, N_dn uniform in 4..8; rings take Ns uniform in 12..16 at half
    filling (N_up = ceil(Ns/2), N_dn = floor(Ns/2)); U uniform in [0, 12]; t=1;
    exponential inter-arrival times at `rate_per_s`.  Returns (arrival_s, Problem)."""
    rng = np.random.default_rng(seed + 7919)
    t_arr, out = 0.0, []
    for i in range(count):
        t_arr += float(rng.exponential(1.0 / rate_per_s))
        fam = int(rng.integers(0, 3))
        U = float(rng.uniform(0.0, 12.0))
        if fam == 0:
            nu, nd = int(rng.integers(4, 9)), int(rng.integers(4, 9))
            p = problem("req%04d_sq3x4_%du%dd" % (i, nu, nd), 12, torus(3, 4), nu, nd, 1.0, U, seed + i)
        elif fam == 1:
            nu, nd = int(rng.integers(4, 9)), int(rng.integers(4, 9))
            p = problem("req%04d_sq4x4_%du%dd" % (i, nu, nd), 16, torus(4, 4), nu, nd, 1.0, U, seed + i)
        else:
            ns = int(rng.integers(12, 17))
            p = problem("req%04d_ring%d" % (i, ns), ns, ring(ns), (ns + 1) // 2, ns // 2, 1.0, U, seed + i)
        out.append((t_arr, p))
    return out


def random_vector(dim: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded uniform[-1, 1) vector (for H.v parity inputs)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=dim).astype(dtype)
