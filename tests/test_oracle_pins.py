"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test names the part of Siro & Harju (arXiv:1204.3425) or the piece of
mathematics it checks against: the paper's worked examples (golden fixtures),
closed forms, symmetries, library eigen-solvers on tiny cases and an
independent second-quantized brute force.
"""
import math

import numpy as np
import pytest

import oracle
import workload
from conftest import golden_rows
from second_quantized import dense_hamiltonian

RNG = np.random.default_rng(20120416)


def _e0_oracle(ns, edges, nu, nd, t, U, seed=workload.BASE_SEED, tol=1e-13, max_iter=400):
    m = oracle.Model(ns, edges, nu, nd, t, U)
    f1 = oracle.start_vector(seed, m.dim)
    return m.lanczos(f1, tol=tol, max_iter=max_iter)["E0"]


# ------------------------------------------------------------------ Sec. 2.1

def test_up_configuration_list():
    """Sec. 2.1: the ordered 4-site, 2-electron configurations."""
    want = [int(r[0], 2) for r in golden_rows("up_configs_4_2.txt")]
    assert list(oracle.basis(4, 2)) == want


def test_table1_labels():
    """Sec. 2.1, Table 1: i_up, i_dn and J for Ns=4, N_up=2, N_dn=3."""
    ups, dns = oracle.basis(4, 2), oracle.basis(4, 3)
    m = oracle.Model(4, workload.ring(4), 2, 3)
    assert m.dim_dn == math.comb(4, 3) == 4
    for up, dn, iu, idn, J in golden_rows("table1_labels.txt"):
        assert oracle.position(ups, int(up, 2)) == int(iu)
        assert oracle.position(dns, int(dn, 2)) == int(idn)
        assert int(iu) * m.dim_dn + int(idn) == int(J)


def test_absent_word_has_no_position():
    assert oracle.position(oracle.basis(4, 2), 0b0111) == -1


@pytest.mark.parametrize("ns", range(1, 13))
def test_dimension_closed_form(ns):
    """Sec. 2.1: dim H = C(Ns, N_up) C(Ns, N_dn)."""
    for nu in range(ns + 1):
        assert len(oracle.basis(ns, nu)) == math.comb(ns, nu)
    for nu, nd in [(0, 0), (ns // 2, (ns + 1) // 2), (ns, ns // 3)]:
        m = oracle.Model(ns, workload.ring(ns) if ns > 1 else [], nu, nd)
        assert m.dim == math.comb(ns, nu) * math.comb(ns, nd)


def test_quoted_sector_dimensions():
    """Sec. 2.1: the half-filled dimensions printed for 12, 14 and 16 sites."""
    for ns, dim, rel in golden_rows("sector_dims.txt"):
        ns, dim, rel = int(ns), float(dim), float(rel)
        d = len(oracle.basis(ns, ns // 2)) ** 2
        assert abs(d - dim) <= rel * dim + 0.5


def test_worked_hop_elements():
    """Sec. 2.1: <2|H|6> has magnitude t, <3|H|6> = 0, <6|H|22> = t, <0|H|3> = -t
    on the 4-site periodic ring (t = 1, U = 0 so H = H_hop)."""
    H = oracle.Model(4, workload.ring(4), 2, 3, t=1.0, U=0.0).dense()
    for r, c, rel, v in golden_rows("hop_elements_ring4.txt"):
        got = H[int(r), int(c)]
        if rel == "abs":
            assert abs(got) == float(v)
        else:
            assert got == float(v)
    # the sign the paper leaves out follows from the same rule: no electron between sites 1 and 2
    assert H[2, 6] == -1.0


SMALL_LATTICES = [
    ("ring2", 2, workload.ring(2)),
    ("ring3", 3, workload.ring(3)),
    ("ring4", 4, workload.ring(4)),
    ("ring5", 5, workload.ring(5)),
    ("ring6", 6, workload.ring(6)),
    ("chain5", 5, workload.chain(5)),
    ("torus2x3", 6, workload.torus(2, 3)),
    ("torus3x2", 6, workload.torus(3, 2)),
]


@pytest.mark.parametrize("name,ns,edges", SMALL_LATTICES)
def test_hamiltonian_matches_second_quantized(name, ns, edges):
    """The oracle's H (signs, J order, diagonal) equals a brute force that applies
    the anticommutation relations of Sec. 1 operator by operator."""
    for nu in range(ns + 1):
        for nd in range(ns + 1):
            if math.comb(ns, nu) * math.comb(ns, nd) > 400:
                continue
            t, U = 1.0 + 0.25 * nu, 3.0 - 0.5 * nd
            ref = dense_hamiltonian(ns, edges, nu, nd, t, U)
            got = oracle.Model(ns, edges, nu, nd, t, U).dense()
            assert np.array_equal(got, ref), (name, nu, nd)


def test_apply_rows_matches_apply():
    m = oracle.Model(6, workload.torus(2, 3), 3, 2, 1.0, 5.0)
    x = RNG.uniform(-1, 1, m.dim)
    rows = RNG.integers(0, m.dim, 50)
    assert np.array_equal(m.apply_rows(x, rows), m.apply(x)[rows])


@pytest.mark.parametrize("ns,n", [(4, 2), (6, 3), (8, 4), (10, 3), (12, 6)])
def test_table_size_closed_form(ns, n):
    """Each bond hops in one direction for every configuration in which exactly
    one of its ends is occupied: nnz(H_sigma) = 2 |E| C(Ns-2, N-1)."""
    edges = workload.ring(ns)
    m = oracle.Model(ns, edges, n, n)
    states, rs, col, val = m.table(0)
    assert len(col) == 2 * len(edges) * math.comb(ns - 2, n - 1)
    # H_sigma is symmetric: the reverse hop has the same element
    entries = {}
    for r in range(len(states)):
        for k in range(rs[r], rs[r + 1]):
            entries[(r, int(col[k]))] = val[k]
    for (r, c), v in entries.items():
        assert entries[(c, r)] == v


def test_trace_closed_form():
    """Tr H = U Ns C(Ns-1, N_up-1) C(Ns-1, N_dn-1): each site is doubly occupied
    in that many basis states."""
    for ns, edges, nu, nd, U in [(6, workload.ring(6), 3, 2, 2.5), (8, workload.torus(2, 4), 3, 4, 4.0)]:
        d = oracle.Model(ns, edges, nu, nd, 1.0, U).diagonal()
        assert d.sum() == pytest.approx(U * ns * math.comb(ns - 1, nu - 1) * math.comb(ns - 1, nd - 1), rel=1e-15)


# ------------------------------------------------------------------ start vector

def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea & Flood 2014), reference implementation seeded
    with 0: its first three outputs."""
    assert oracle.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 2) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(0, 3) == 0x06C45D188009454F


def test_start_vector_is_uniform_and_unit():
    f_raw = oracle.start_vector(7, 200000, normalise=False)
    assert f_raw.min() >= -1.0 and f_raw.max() < 1.0
    assert abs(f_raw.mean()) < 0.01 and abs(f_raw.var() - 1.0 / 3.0) < 0.01
    # element J comes from counter J+1: u = top 53 bits / 2^53
    u = (oracle.splitmix64(7, 1) >> 11) / 2.0**53
    assert f_raw[0] == 2.0 * u - 1.0
    f = oracle.start_vector(7, 1000)
    assert abs(np.linalg.norm(f) - 1.0) < 1e-15


# ------------------------------------------------------------------ T eigensolver

def test_tridiag_min_matches_library():
    """Lowest eigenvalue of a symmetric tridiagonal T (eq. Tmatrix) against LAPACK."""
    for m in [1, 2, 3, 7, 50, 200]:
        a = RNG.normal(size=m)
        boff = np.concatenate([[0.0], RNG.uniform(0.1, 2.0, size=m - 1)])
        T = np.diag(a) + np.diag(boff[1:], 1) + np.diag(boff[1:], -1)
        ref = np.linalg.eigvalsh(T)[0]
        assert oracle.tridiag_min(a, boff) == pytest.approx(ref, abs=1e-13 * max(1, np.abs(T).max()))


def test_tridiag_min_closed_form():
    """a_j = 0, b_j = 1: eigenvalues 2 cos(k pi / (m+1)), lowest -2 cos(pi/(m+1))."""
    for m in [2, 10, 100, 300]:
        got = oracle.tridiag_min(np.zeros(m), np.ones(m))
        assert got == pytest.approx(-2.0 * math.cos(math.pi / (m + 1)), abs=2e-15)


def test_tridiag_vec():
    m = 40
    a = RNG.normal(size=m)
    boff = np.concatenate([[0.0], RNG.uniform(0.1, 2.0, size=m - 1)])
    T = np.diag(a) + np.diag(boff[1:], 1) + np.diag(boff[1:], -1)
    w, V = np.linalg.eigh(T)
    y = oracle.tridiag_vec(a, boff, oracle.tridiag_min(a, boff))
    assert y[0] > 0 and abs(np.linalg.norm(y) - 1) < 1e-14
    assert abs(abs(y @ V[:, 0]) - 1.0) < 1e-12
    assert np.linalg.norm(T @ y - w[0] * y) < 1e-12


# ------------------------------------------------------------------ E0 pins

@pytest.mark.parametrize("name,ns,edges", SMALL_LATTICES)
def test_e0_matches_dense_diagonalisation(name, ns, edges):
    """Lanczos E0 (Alg. 1 + Sturm bisection) equals the lowest eigenvalue of the
    brute-force H for every sector of the tiny lattices."""
    for nu in range(ns + 1):
        for nd in range(ns + 1):
            if math.comb(ns, nu) * math.comb(ns, nd) > 400:
                continue
            U = 4.0
            ref = np.linalg.eigvalsh(dense_hamiltonian(ns, edges, nu, nd, 1.0, U))[0]
            got = _e0_oracle(ns, edges, nu, nd, 1.0, U)
            assert got == pytest.approx(ref, rel=1e-10, abs=1e-10), (name, nu, nd)


def test_ring8_half_filling_dense():
    """The 4,900-dim ring of 8 sites, U=4: Lanczos E0 equals LAPACK's lowest eigenvalue."""
    p = workload.ring8()
    H = dense_hamiltonian(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    w, V = np.linalg.eigh(H)
    ref = w[0]
    assert w[1] - w[0] > 0.1  # nondegenerate ground state: psi is unique up to sign
    m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    r = m.lanczos(oracle.start_vector(p.seed, m.dim), tol=1e-12, max_iter=300, want_psi=True)
    assert r["converged"] == 1
    assert r["E0"] == pytest.approx(ref, rel=1e-10)
    assert r["residual"] < 1e-5
    assert r["rayleigh"] == pytest.approx(ref, rel=1e-12)
    assert abs(r["psi"] @ V[:, 0]) > 1.0 - 1e-10
    assert abs(np.linalg.norm(r["psi"]) - 1.0) < 1e-14


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 10.0])
@pytest.mark.parametrize("t", [1.0, 0.5])
def test_dimer_closed_form(U, t):
    """Two sites, one bond, one electron of each spin: E0 = U/2 - sqrt(U^2/4 + 4 t^2)."""
    got = _e0_oracle(2, [(0, 1)], 1, 1, t, U)
    assert got == pytest.approx(U / 2 - math.sqrt(U * U / 4 + 4 * t * t), rel=1e-12, abs=1e-14)


def _lowest_levels_sum(adj_eigs, n):
    return float(np.sort(adj_eigs)[:n].sum())


@pytest.mark.parametrize("ns,nu,nd", [(6, 3, 3), (8, 3, 2), (10, 5, 4), (12, 4, 4)])
def test_free_ring_closed_form(ns, nu, nd):
    """U = 0 on a ring: E0 = sum of the lowest N_up and the lowest N_dn levels
    -2t cos(2 pi k / Ns)."""
    t = 1.0
    lev = np.array([-2 * t * math.cos(2 * math.pi * k / ns) for k in range(ns)])
    ref = _lowest_levels_sum(lev, nu) + _lowest_levels_sum(lev, nd)
    assert _e0_oracle(ns, workload.ring(ns), nu, nd, t, 0.0) == pytest.approx(ref, rel=1e-10)


def test_free_torus_closed_form():
    """U = 0 on a 3x4 periodic lattice: levels -2t (cos kx + cos ky)."""
    lx, ly, nu, nd, t = 3, 4, 3, 4, 1.0
    lev = np.array([-2 * t * (math.cos(2 * math.pi * i / lx) + math.cos(2 * math.pi * j / ly))
                    for i in range(lx) for j in range(ly)])
    ref = _lowest_levels_sum(lev, nu) + _lowest_levels_sum(lev, nd)
    assert _e0_oracle(lx * ly, workload.torus(lx, ly), nu, nd, t, 0.0) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("ns,nu,nd", [(6, 3, 3), (6, 4, 5), (8, 2, 6)])
def test_atomic_limit(ns, nu, nd):
    """t = 0: E0 = U max(0, N_up + N_dn - Ns) for U >= 0."""
    U = 3.0
    assert _e0_oracle(ns, workload.ring(ns), nu, nd, 0.0, U) == pytest.approx(U * max(0, nu + nd - ns), abs=1e-12)


def test_symmetries():
    """Spin flip; particle-hole on a bipartite lattice; t -> -t; scaling."""
    ns, edges, U = 8, workload.ring(8), 4.0
    e = {}
    for nu, nd in [(2, 3), (3, 2), (6, 5), (5, 6)]:
        e[(nu, nd)] = _e0_oracle(ns, edges, nu, nd, 1.0, U)
    assert e[(2, 3)] == pytest.approx(e[(3, 2)], rel=1e-11)
    # particle-hole: E(Nu, Nd) - E(Ns-Nu, Ns-Nd) = U (Nu + Nd - Ns)
    assert e[(2, 3)] - e[(6, 5)] == pytest.approx(U * (2 + 3 - ns), rel=1e-10)
    assert e[(3, 2)] - e[(5, 6)] == pytest.approx(U * (3 + 2 - ns), rel=1e-10)
    # t -> -t on a bipartite lattice, E(lambda t, lambda U) = lambda E(t, U)
    assert _e0_oracle(ns, edges, 3, 4, -1.0, U) == pytest.approx(_e0_oracle(ns, edges, 3, 4, 1.0, U), rel=1e-11)
    assert _e0_oracle(ns, edges, 3, 4, 2.5, 2.5 * U) == pytest.approx(2.5 * _e0_oracle(ns, edges, 3, 4, 1.0, U), rel=1e-11)


# ------------------------------------------------------------------ Lanczos recurrence

def test_lanczos_recurrence_reproduces_tridiagonal_projection():
    """Alg. 1 in exact-Krylov regime: re-running the recurrence with numpy on the
    brute-force H gives the same a_j, b_{j+1}; the Lanczos basis spans the Krylov
    space (Sec. 2.2)."""
    ns, edges, nu, nd = 6, workload.torus(2, 3), 3, 3
    H = dense_hamiltonian(ns, edges, nu, nd, 1.0, 2.0)
    m = oracle.Model(ns, edges, nu, nd, 1.0, 2.0)
    f1 = oracle.start_vector(99, m.dim)
    r = m.lanczos(f1, tol=0.0 + 1e-300, max_iter=12)
    f_prev, f, bj = np.zeros(m.dim), f1.copy(), 0.0
    for j in range(r["n_iter"]):
        q = H @ f - bj * f_prev
        a = q @ f
        q = q - a * f
        b = math.sqrt(q @ q)
        assert a == pytest.approx(r["a"][j], rel=1e-12, abs=1e-13)
        assert b == pytest.approx(r["b"][j], rel=1e-10)
        f_prev, f, bj = f, q / b, b


def test_breakdown_on_one_dimensional_sector():
    """N = 0 and N = Ns give a 1x1 H: b_2 = 0 stops Alg. 1 after one step."""
    m = oracle.Model(4, workload.ring(4), 4, 0, 1.0, 2.0)
    assert m.dim == 1
    r = m.lanczos(np.ones(1), tol=1e-12, max_iter=10, want_psi=True)
    assert r["n_iter"] == 1 and r["converged"] == 2
    assert abs(r["E0"]) < 1e-300 and r["residual"] < 1e-300


# ------------------------------------------------------------------ lowest states (Sec. 2.2)

def _check_eigvecs(m, w, V):
    """Rows of V are orthonormal and H v = w v for each."""
    assert np.abs(V @ V.T - np.eye(len(w))).max() < 1e-12
    for e, v in zip(w, V):
        assert np.linalg.norm(m.apply(v) - e * v) < 1e-11 * max(1.0, abs(e))


@pytest.mark.parametrize("U", [0.0, 3.7])
@pytest.mark.parametrize("t", [1.3, -0.6])
def test_lowest_states_dimer_full_spectrum(U, t):
    """Two sites, one electron of each spin: the four levels are the triplet 0,
    the antisymmetric doubly-occupied state U, and (U -+ sqrt(U^2 + 16 t^2)) / 2."""
    m = oracle.Model(2, [(0, 1)], 1, 1, t, U)
    w, V = m.lowest_states(4)
    r = math.sqrt(U * U + 16 * t * t)
    want = np.sort([0.0, U, (U - r) / 2, (U + r) / 2])
    assert np.allclose(w, want, rtol=0, atol=1e-13)
    _check_eigvecs(m, w, V)


def _atomic_spectrum(ns, nu, nd, U):
    """t = 0: level U d with multiplicity C(Ns, d) C(Ns-d, Nu-d) C(Ns-Nu, Nd-d)
    (choose the doubly occupied sites, then the lone up spins, then the lone
    down spins among the sites without an up spin)."""
    out = []
    for d in range(0, min(nu, nd) + 1):
        mult = math.comb(ns, d) * math.comb(ns - d, nu - d) * math.comb(ns - nu, nd - d)
        out += [U * d] * mult
    return np.sort(np.array(out, dtype=float))


@pytest.mark.parametrize("ns,nu,nd", [(4, 3, 3), (5, 3, 2), (6, 3, 3)])
def test_lowest_states_atomic_limit_multiplicities(ns, nu, nd):
    U = 2.5
    m = oracle.Model(ns, workload.ring(ns), nu, nd, 0.0, U)
    ref = _atomic_spectrum(ns, nu, nd, U)
    assert len(ref) == m.dim
    w, V = m.lowest_states(m.dim)
    assert np.array_equal(w.round(12), ref.round(12))
    _check_eigvecs(m, w, V)


def _free_spectrum(levels, nu, nd):
    """U = 0: every eigenvalue is a sum over N_up distinct levels plus a sum over
    N_dn distinct levels (Slater determinants of each spin)."""
    import itertools
    su = [sum(c) for c in itertools.combinations(levels, nu)]
    sd = [sum(c) for c in itertools.combinations(levels, nd)]
    return np.sort(np.add.outer(su, sd).ravel())


@pytest.mark.parametrize("kind,ns,nu,nd", [("ring", 6, 2, 3), ("ring", 7, 3, 3), ("chain", 6, 3, 2)])
def test_lowest_states_free_fermion_spectrum(kind, ns, nu, nd):
    """U = 0: ring levels -2t cos(2 pi k / Ns); open-chain levels -2t cos(pi k / (Ns+1))."""
    t = 0.8
    if kind == "ring":
        edges = workload.ring(ns)
        lev = [-2 * t * math.cos(2 * math.pi * k / ns) for k in range(ns)]
    else:
        edges = workload.chain(ns)
        lev = [-2 * t * math.cos(math.pi * k / (ns + 1)) for k in range(1, ns + 1)]
    m = oracle.Model(ns, edges, nu, nd, t, 0.0)
    ref = _free_spectrum(lev, nu, nd)
    k = min(40, m.dim)
    w, V = m.lowest_states(k)
    assert np.allclose(w, ref[:k], rtol=0, atol=1e-11)
    _check_eigvecs(m, w, V)


def test_lowest_states_trace_and_ordering():
    """Interacting case: the full spectrum is ascending and sums to the trace,
    U times the number of doubly occupied sites summed over the basis,
    sum_d d * mult(d) with the multiplicities of the atomic limit."""
    ns, nu, nd, U = 6, 3, 2, 4.0
    m = oracle.Model(ns, workload.torus(2, 3), nu, nd, 1.0, U)
    w, V = m.lowest_states(m.dim)
    assert np.all(np.diff(w) >= 0)
    ref = _atomic_spectrum(ns, nu, nd, U).sum()
    assert w.sum() == pytest.approx(ref, rel=1e-12)
    _check_eigvecs(m, w, V)


# ------------------------------------------------------------------ site observables (Sec. 1, eq. H)

def _ground(ns, edges, nu, nd, t, U):
    m = oracle.Model(ns, edges, nu, nd, t, U)
    w, V = m.lowest_states(2)
    return m, w, V[0]


@pytest.mark.parametrize("U", [0.5, 4.0])
@pytest.mark.parametrize("kind", ["torus2x3", "chain6"])
def test_double_occupancy_is_dE0_dU(kind, U):
    """Hellmann-Feynman: for a non-degenerate ground state dE0/dU = <sum_i n_i,up n_i,dn>,
    checked against a central difference of the dense E0."""
    ns, edges = (6, workload.torus(2, 3)) if kind == "torus2x3" else (6, workload.chain(6))
    nu, nd, t = (3, 3, 1.0) if kind == "torus2x3" else (3, 2, 1.0)
    m, w, v = _ground(ns, edges, nu, nd, t, U)
    assert w[1] - w[0] > 1e-3  # non-degenerate
    d = 1e-4
    e = [oracle.Model(ns, edges, nu, nd, t, U + s * d).lowest_states(1)[0][0] for s in (-1, 1)]
    assert m.observables(v)["docc"] == pytest.approx((e[1] - e[0]) / (2 * d), abs=1e-7)


@pytest.mark.parametrize("U", [0.0, 2.0, 9.0])
def test_double_occupancy_dimer_closed_form(U):
    """Dimer ground state: D = (1 - U / sqrt(U^2 + 16 t^2)) / 2, the U-derivative of
    E0 = (U - sqrt(U^2 + 16 t^2)) / 2."""
    t = 0.7
    m, _, v = _ground(2, [(0, 1)], 1, 1, t, U)
    o = m.observables(v)
    assert o["docc"] == pytest.approx((1 - U / math.sqrt(U * U + 16 * t * t)) / 2, abs=1e-13)
    assert np.allclose(o["dens"], 0.5, atol=1e-13)


def test_free_chain_densities_and_factorisation():
    """U = 0 on an open chain (non-degenerate ground state): <n_i sigma> = sum over the
    N_sigma lowest orbitals of phi_k(i)^2, phi_k(i) = sqrt(2/(L+1)) sin(pi k (i+1) / (L+1)),
    and up and down electrons are independent: <n_i,up n_j,dn> = <n_i,up><n_j,dn>."""
    L, nu, nd = 7, 3, 2
    m, w, v = _ground(L, workload.chain(L), nu, nd, 1.0, 0.0)
    assert w[1] - w[0] > 1e-3
    o = m.observables(v)
    phi = lambda k, i: math.sqrt(2 / (L + 1)) * math.sin(math.pi * k * (i + 1) / (L + 1))
    for s, n in ((0, nu), (1, nd)):
        ref = [sum(phi(k, i) ** 2 for k in range(1, n + 1)) for i in range(L)]
        assert np.allclose(o["dens"][s], ref, atol=1e-12)
    assert np.allclose(o["corr"][2], np.outer(o["dens"][0], o["dens"][1]), atol=1e-12)


def test_atomic_limit_has_no_double_occupancy():
    """t = 0, U > 0, N_up + N_dn <= Ns: every ground state has no doubly occupied site."""
    m = oracle.Model(6, workload.ring(6), 3, 2, 0.0, 3.0)
    w, V = m.lowest_states(5)
    for v in V:
        assert m.observables(v)["docc"] == 0.0


def test_observable_sum_rules():
    """sum_i <n_i s> = N_s; <n_i s n_i s> = <n_i s>; sum_j <n_i a n_j b> = N_b <n_i a>;
    the (up, up) and (dn, dn) blocks are symmetric; an unnormalised psi gives the same values."""
    ns, nu, nd = 6, 3, 2
    m = oracle.Model(ns, workload.torus(2, 3), nu, nd, 1.0, 3.0)
    v = RNG.uniform(-1, 1, m.dim)  # any state, not an eigenvector
    o = m.observables(v)
    assert o["dens"][0].sum() == pytest.approx(nu, abs=1e-12)
    assert o["dens"][1].sum() == pytest.approx(nd, abs=1e-12)
    for k, (a, b, nb) in enumerate(((0, 0, nu), (1, 1, nd), (0, 1, nd))):
        C = o["corr"][k]
        assert np.allclose(C.sum(axis=1), nb * o["dens"][a], atol=1e-12)
        if a == b:
            assert np.allclose(np.diag(C), o["dens"][a], atol=1e-13)
            assert np.allclose(C, C.T, atol=1e-13)
    assert np.allclose(o["corr"][2].sum(axis=0), nu * o["dens"][1], atol=1e-12)
    o2 = m.observables(3.0 * v)
    assert np.allclose(o2["corr"], o["corr"], atol=1e-14) and o2["docc"] == pytest.approx(o["docc"], abs=1e-14)


# ------------------------------------------------------------------ time evolution exp(-i H t)

def test_propagate_single_particle_ring_closed_form():
    """One up electron on an L-site ring, U irrelevant: starting on site 0 the amplitude
    on site j at time T is (1/L) sum_k exp(i k j) exp(2 i t T cos k), k = 2 pi n / L."""
    L, t, T = 7, 0.9, 1.7
    m = oracle.Model(L, workload.ring(L), 1, 0, t, 5.0)
    states = oracle.basis(L, 1)
    psi0 = np.zeros(m.dim, dtype=complex)
    psi0[oracle.position(states, 1)] = 1.0
    got = m.propagate(psi0, T)
    for j in range(L):
        ref = sum(np.exp(1j * k * j) * np.exp(2j * t * T * math.cos(k))
                  for k in (2 * math.pi * n / L for n in range(L))) / L
        assert abs(got[oracle.position(states, 1 << j)] - ref) < 1e-12


def test_propagate_atomic_limit_phases():
    """t = 0: each configuration only picks up the phase exp(-i U d_J T), d_J its
    number of doubly occupied sites."""
    ns, nu, nd, U, T = 5, 3, 2, 1.3, 2.2
    m = oracle.Model(ns, workload.ring(ns), nu, nd, 0.0, U)
    d = m.diagonal() / U
    psi0 = RNG.uniform(-1, 1, m.dim) + 1j * RNG.uniform(-1, 1, m.dim)
    assert np.allclose(m.propagate(psi0, T), np.exp(-1j * U * d * T) * psi0, atol=1e-13)


def test_propagate_eigenstate_phase_group_and_unitarity():
    """An eigenvector only gains exp(-i E T); exp(-iH a) exp(-iH b) = exp(-iH (a+b));
    the norm and <H> are conserved; T = 0 is the identity."""
    m = oracle.Model(6, workload.torus(2, 3), 3, 3, 1.0, 3.0)
    w, V = m.lowest_states(1)
    assert np.allclose(m.propagate(V[0], 0.8), np.exp(-0.8j * w[0]) * V[0], atol=1e-12)
    psi0 = RNG.uniform(-1, 1, m.dim) + 1j * RNG.uniform(-1, 1, m.dim)
    a = m.propagate(m.propagate(psi0, 0.3), 0.45)
    assert np.allclose(a, m.propagate(psi0, 0.75), atol=1e-12)
    assert np.linalg.norm(a) == pytest.approx(np.linalg.norm(psi0), rel=1e-13)
    e = lambda v: (np.vdot(v, m.apply(v.real) + 1j * m.apply(v.imag)) / np.vdot(v, v)).real
    assert e(a) == pytest.approx(e(psi0), rel=1e-12)
    assert np.allclose(m.propagate(psi0, 0.0), psi0, atol=1e-14)


# ------------------------------------------------------------------ per-bond amplitudes t_ij

@pytest.mark.parametrize("name,ns,edges", SMALL_LATTICES[2:])
def test_bond_amplitudes_match_second_quantized(name, ns, edges):
    """eq. H with t_ij in place of t (Sec. 2.1: any lattice): the oracle's H equals
    the operator-by-operator brute force for random per-bond amplitudes."""
    g = np.random.default_rng(len(edges) * 31 + ns)
    amps = g.uniform(-2, 2, len(edges))
    for nu, nd in [(1, 1), (2, 1), (ns // 2, (ns + 1) // 2)]:
        if math.comb(ns, nu) * math.comb(ns, nd) > 400:
            continue
        ref = dense_hamiltonian(ns, edges, nu, nd, amps, 1.7)
        got = oracle.Model(ns, edges, nu, nd, amps, 1.7).dense()
        assert np.allclose(got, ref, rtol=0, atol=1e-15), (name, nu, nd)


def test_bond_amplitudes_uniform_is_the_scalar_model():
    m1 = oracle.Model(6, workload.torus(2, 3), 3, 2, 1.3, 4.0)
    m2 = oracle.Model(6, workload.torus(2, 3), 3, 2, [1.3] * len(workload.torus(2, 3)), 4.0)
    assert np.array_equal(m1.dense(), m2.dense())


def test_bond_amplitudes_ssh_single_particle_band():
    """One electron on an even ring with alternating amplitudes t1, t2 (two-site
    unit cell): levels +-|t1 + t2 exp(i q)|, q = 2 pi n / (L/2)."""
    L, t1, t2 = 10, 1.0, 0.45
    edges = workload.ring(L)
    amps = [t1 if (min(i, j) % 2 == 0 and abs(i - j) == 1) else t2 for (i, j) in edges]
    # the wrap bond (0, L-1) joins cells: it carries t2
    m = oracle.Model(L, edges, 1, 0, amps, 3.0)
    w = np.linalg.eigvalsh(m.dense())
    qs = [2 * math.pi * n / (L // 2) for n in range(L // 2)]
    ref = np.sort([s * abs(t1 + t2 * np.exp(1j * q)) for q in qs for s in (1, -1)])
    assert np.allclose(w, ref, atol=1e-12)


def test_bond_amplitude_sign_gauge():
    """Flipping the sign of every bond leaving one sublattice site of a bipartite
    lattice is a gauge transformation (c_i -> -c_i on that site): the spectrum stays."""
    ns, edges = 8, workload.ring(8)
    g = np.random.default_rng(5)
    amps = g.uniform(0.5, 1.5, len(edges))
    flip = np.array([-a if 3 in e else a for a, e in zip(amps, edges)])
    w1 = np.linalg.eigvalsh(oracle.Model(ns, edges, 2, 2, amps, 2.0).dense())
    w2 = np.linalg.eigvalsh(oracle.Model(ns, edges, 2, 2, flip, 2.0).dense())
    assert np.allclose(w1, w2, atol=1e-11)
