"""GPU parity with one hopping amplitude per bond (hubbard_build_bonds: eq. H
with t_ij for t) against the oracle's per-bond model.

H.v: the same bound as the one-amplitude case (a sum of at most 1 + w_up + w_dn
terms in a different order): max|y - y_ref| <= 1e-13 max|y_ref| in FP64 and
the FP32 bound n u sum|terms| in mixed precision.  E0: 1e-10 relative (FP64),
1e-6 (mixed), against the oracle's Lanczos from the same start vector.  The
per-bond handle with at most four amplitude classes runs the two-pass kernels
(class bits in the row-pass groups and the up-spin entries), one with more
runs the one-pass kernel, with its row staged in LDS and (rows wider than LDS)
not staged; all of these are covered.
"""
import numpy as np
import pytest

import oracle
import workload

torch = pytest.importorskip("torch")
hb = pytest.importorskip("paper_1204_3425_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _tt_prime_torus(lx, ly, t1, t2):
    """Square lattice with nearest-neighbour bonds t1 and one diagonal per plaquette t2."""
    nn = workload.torus(lx, ly)
    diag = []
    for y in range(ly):
        for x in range(lx):
            a, b = x + lx * y, (x + 1) % lx + lx * ((y + 1) % ly)
            if a != b and (min(a, b), max(a, b)) not in {(min(i, j), max(i, j)) for i, j in nn + diag}:
                diag.append((a, b))
    return nn + diag, [t1] * len(nn) + [t2] * len(diag)


CASES = [
    # name, sites, edges, amplitudes, n_up, n_dn, U
    ("ring8_random", 8, workload.ring(8), np.random.default_rng(1).uniform(-1.5, 1.5, 8), 4, 3, 3.0),
    ("torus3x4_tprime", 12, *_tt_prime_torus(3, 4, 1.0, -0.35), 3, 3, 6.0),
    ("chain10_ssh", 10, workload.chain(10), [1.0 if i % 2 == 0 else 0.4 for i in range(9)], 5, 5, 2.0),
    # rows of 48,620 elements (18 sites, 9 down): wider than LDS, the kernel reads x directly
    ("ring18_1u9d", 18, workload.ring(18), np.random.default_rng(2).uniform(0.5, 1.5, 18), 1, 9, 4.0),
    # four amplitude classes (the most the two-pass kernels take) and five (one-pass)
    ("ring10_4classes", 10, workload.ring(10), [0.5, 0.8, -1.1, 1.4] * 2 + [0.5, 0.8], 4, 4, 3.0),
    ("ring10_5classes", 10, workload.ring(10), [0.5, 0.8, -1.1, 1.4, 0.9] * 2, 4, 4, 3.0),
]


def _two_pass(h):
    """The two-pass kernels run with padded rows (ld_pref a multiple of 64 above
    dim_dn), the one-pass kernel with dense ones (ld_pref = dim_dn)."""
    return hb.hubbard_info(h)["ld_pref"] != h.dim_dn


def test_bonds_kernel_choice():
    """Up to four amplitude classes take the two-pass kernels, more take the one-pass kernel."""
    want = {"ring8_random": False, "torus3x4_tprime": True, "chain10_ssh": True, "ring18_1u9d": False,
            "ring10_4classes": True, "ring10_5classes": False}
    for name, sites, edges, amps, nu, nd, U in CASES:
        h = hb.hubbard_build_bonds(sites, edges, amps, nu, nd, U)
        assert _two_pass(h) == want[name], name


@pytest.mark.parametrize("name,sites,edges,amps,nu,nd,U", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
def test_bonds_apply_parity(name, sites, edges, amps, nu, nd, U, precision):
    _say("apply", name, precision)
    h = hb.hubbard_build_bonds(sites, edges, amps, nu, nd, U)
    m = oracle.Model(sites, edges, nu, nd, amps, U)
    x = workload.random_vector(m.dim, workload.BASE_SEED)
    ref = m.apply(x)
    hb.hubbard_set_precision(h, precision)
    dt = torch.float64 if precision == hb.HUBBARD_FP64 else torch.float32
    xd = torch.from_numpy(x).to(DEV, dt)
    yd = torch.empty_like(xd)
    hb.hubbard_apply(h, xd, yd)
    torch.cuda.synchronize()
    y = yd.double().cpu().numpy()
    if precision == hb.HUBBARD_FP64:
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    else:
        # FP32 accumulation of FP32 inputs: n u sum|terms| with n = 1 + w_up + w_dn
        # terms, each hop at most max|t| max|x| and the diagonal U D_J x_J at most
        # |U| min(N_up, N_dn) max|x|
        info = hb.hubbard_info(h)
        w = info["w_up"] + info["w_dn"]
        xf = xd.double().cpu().numpy()  # the rounded input the GPU saw
        S = (np.abs(amps).max() * w + abs(U) * min(nu, nd)) * np.abs(xf).max()
        assert np.abs(y - m.apply(xf)).max() <= (1 + w) * 2.0 ** -24 * S


@pytest.mark.parametrize("name,sites,edges,amps,nu,nd,U", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_bonds_lanczos_parity(name, sites, edges, amps, nu, nd, U):
    _say("lanczos", name)
    h = hb.hubbard_build_bonds(sites, edges, amps, nu, nd, U)
    m = oracle.Model(sites, edges, nu, nd, amps, U)
    ref = m.lanczos(oracle.start_vector(workload.BASE_SEED, m.dim), tol=1e-12, max_iter=400)
    psi = torch.zeros(h.dim, dtype=torch.float64, device=DEV)
    r = hb.hubbard_lanczos_ex(h, tol=1e-12, max_iter=400, precision=hb.HUBBARD_FP64, seed=workload.BASE_SEED,
                              psi=psi)
    assert r["E0"] == pytest.approx(ref["E0"], rel=1e-10)
    assert np.allclose(r["a"][:20], ref["a"][:20], rtol=1e-12, atol=1e-12)
    assert r["residual"] <= 1e-4
    rm = hb.hubbard_lanczos_ex(h, tol=1e-10, max_iter=400, precision=hb.HUBBARD_MIXED, seed=workload.BASE_SEED)
    assert abs(rm["E0"] - ref["E0"]) <= 1e-6 * max(1.0, abs(ref["E0"]))


def test_bonds_uniform_list_is_the_plain_handle():
    """All amplitudes equal: the same handle as hubbard_build, bit for bit (two-pass kernels)."""
    p = workload.ring8()
    h1 = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    h2 = hb.hubbard_build_bonds(p.sites, p.edges, [p.t] * len(p.edges), p.n_up, p.n_dn, p.U)
    r1 = hb.hubbard_lanczos_ex(h1, tol=1e-12, max_iter=300, precision=hb.HUBBARD_FP64, seed=p.seed)
    r2 = hb.hubbard_lanczos_ex(h2, tol=1e-12, max_iter=300, precision=hb.HUBBARD_FP64, seed=p.seed)
    assert r1["E0"] == r2["E0"] and np.array_equal(r1["a"], r2["a"])


def test_bonds_through_lowest_states_propagate_and_batch():
    """The other entry points run on a per-bond handle: lowest states against the
    dense spectrum, propagation against the dense exponential, and the batch
    call (which runs such a handle unbatched) against the single solve."""
    sites, (edges, amps), nu, nd, U = 9, _tt_prime_torus(3, 3, 1.0, -0.35), 2, 2, 5.0  # dim 1,296
    h = hb.hubbard_build_bonds(sites, edges, amps, nu, nd, U)
    m = oracle.Model(sites, edges, nu, nd, amps, U)
    w = m.lowest_states(3)[0]
    E, _ = hb.hubbard_lowest_states(h, 3, tol=1e-14, max_iter=600, precision=hb.HUBBARD_FP64)
    assert np.all(np.abs(E - w) <= 1e-10 * np.maximum(1.0, np.abs(w)))
    g = np.random.default_rng(3)
    psi0 = g.uniform(-1, 1, m.dim) + 1j * g.uniform(-1, 1, m.dim)
    re = torch.from_numpy(psi0.real.copy()).to(DEV)
    im = torch.from_numpy(psi0.imag.copy()).to(DEV)
    hb.hubbard_propagate(h, re, im, 0.7, 5, 20)
    got = re.cpu().numpy() + 1j * im.cpu().numpy()
    assert np.abs(got - m.propagate(psi0, 0.7)).max() <= 1e-10 * np.linalg.norm(psi0)
    single = hb.hubbard_lanczos_ex(h, tol=1e-12, max_iter=300, precision=hb.HUBBARD_FP64, seed=7)
    hu = hb.hubbard_build(8, workload.ring(8), 3, 3, 1.0, 2.0)
    batch = hb.hubbard_lanczos_batch([h, hu], tol=1e-12, max_iter=300, precision=hb.HUBBARD_FP64, seeds=[7, 7])
    assert batch[0]["E0"] == single["E0"]


@pytest.mark.parametrize("per_bond", [False, True], ids=["one_amplitude", "per_bond"])
def test_rows_of_33_to_64_hops(per_bond):
    """The 4x4 lattice with diagonal bonds, 8 up + 2 down (dim 1.54M): up rows of
    up to 48 hops take the two-line (64-slot) layout of the up-spin pass.  H.v in
    FP64 and FP32 against the oracle, the first 20 Lanczos coefficients of the
    fused step (sectors of 65,536 states and more) against the oracle's from the
    same start vector in FP64 and mixed precision, and the FP64 residual that a
    converged solve reports (the residual epilogue of the same kernels) against
    ||H psi - E0 psi|| from the oracle's H on the returned psi."""
    edges, amps = workload.torus_tprime(4, 4, 1.0, -0.3 if per_bond else 1.0)
    U = 5.0
    h = (hb.hubbard_build_bonds(16, edges, amps, 8, 2, U) if per_bond
         else hb.hubbard_build(16, edges, 8, 2, 1.0, U))
    info = hb.hubbard_info(h)
    assert 32 < info["w_up"] <= 64 and _two_pass(h)
    m = oracle.Model(16, edges, 8, 2, amps if per_bond else 1.0, U)
    x = workload.random_vector(m.dim, workload.BASE_SEED)
    ref = m.apply(x)
    for precision, dt in ((hb.HUBBARD_FP64, torch.float64), (hb.HUBBARD_MIXED, torch.float32)):
        hb.hubbard_set_precision(h, precision)
        xd = torch.from_numpy(x).to(DEV, dt)
        yd = torch.empty_like(xd)
        hb.hubbard_apply(h, xd, yd)
        torch.cuda.synchronize()
        y = yd.double().cpu().numpy()
        tol = 1e-13 if precision == hb.HUBBARD_FP64 else 64 * (1 + info["w_up"] + info["w_dn"]) * 2.0 ** -24
        assert np.abs(y - ref).max() <= tol * np.abs(ref).max(), precision
    f1 = oracle.start_vector(workload.BASE_SEED, m.dim)
    ro = m.lanczos(f1, tol=1e-300, max_iter=20)
    r = hb.hubbard_lanczos_ex(h, tol=-1.0, max_iter=20, precision=hb.HUBBARD_FP64, seed=workload.BASE_SEED)
    assert np.allclose(r["a"], ro["a"], rtol=1e-12, atol=1e-12)
    assert np.allclose(r["b"], ro["b"], rtol=1e-10, atol=1e-12)
    # FP32 vectors: coefficients within a few FP32 ulps of the H.v sums, grown over 20 steps
    rm = hb.hubbard_lanczos_ex(h, tol=-1.0, max_iter=20, precision=hb.HUBBARD_MIXED, seed=workload.BASE_SEED)
    assert np.allclose(rm["a"], ro["a"], rtol=1e-4, atol=1e-4)
    psi = torch.zeros(h.dim, dtype=torch.float64, device=DEV)
    rs = hb.hubbard_lanczos_ex(h, tol=1e-12, max_iter=600, precision=hb.HUBBARD_FP64, seed=workload.BASE_SEED,
                               psi=psi)
    v = psi.cpu().numpy()
    res = np.linalg.norm(m.apply(v) - rs["E0"] * v) / np.linalg.norm(v)
    _say("residual", rs["residual"], "oracle", res, "steps", rs["n_iter"])
    assert 0.0 <= rs["residual"] <= 1e-4
    assert abs(rs["residual"] - res) <= 1e-9 + 1e-6 * res


def test_per_bond_up_rows_over_64_hops():
    """Two amplitude classes on up rows of up to 72 hops (17 sites, each pair
    bonded with probability 0.9, seeded; 8 up + 1 down, 413,270 states): the
    per-bond variant of the variable-width blocked pass.  H.v in FP64 and FP32
    against the oracle's per-bond model, and 20 Lanczos steps of the fused step
    against the oracle's from the same start vector."""
    g = np.random.default_rng(17)
    edges = [(i, j) for i in range(17) for j in range(i + 1, 17) if g.random() < 0.9]
    amps = [1.0 if k % 3 else 0.55 for k in range(len(edges))]
    U = 3.0
    h = hb.hubbard_build_bonds(17, edges, amps, 8, 1, U)
    info = hb.hubbard_info(h)
    assert info["w_up"] > 64 and _two_pass(h)
    m = oracle.Model(17, edges, 8, 1, amps, U)
    x = workload.random_vector(m.dim, workload.BASE_SEED + 1)
    ref = m.apply(x)
    for precision, dt in ((hb.HUBBARD_FP64, torch.float64), (hb.HUBBARD_MIXED, torch.float32)):
        hb.hubbard_set_precision(h, precision)
        xd = torch.from_numpy(x).to(DEV, dt)
        yd = torch.empty_like(xd)
        hb.hubbard_apply(h, xd, yd)
        torch.cuda.synchronize()
        y = yd.double().cpu().numpy()
        if precision == hb.HUBBARD_FP64:
            assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
        else:
            # the FP32 bound of the other per-bond cases: n u sum|terms|
            w = info["w_up"] + info["w_dn"]
            xf = xd.double().cpu().numpy()
            S = (max(amps) * w + U * 1) * np.abs(xf).max()
            assert np.abs(y - m.apply(xf)).max() <= (1 + w) * 2.0 ** -24 * S
    ro = m.lanczos(oracle.start_vector(workload.BASE_SEED, m.dim), tol=1e-300, max_iter=20)
    r = hb.hubbard_lanczos_ex(h, tol=-1.0, max_iter=20, precision=hb.HUBBARD_FP64, seed=workload.BASE_SEED)
    assert np.allclose(r["a"], ro["a"], rtol=1e-12, atol=1e-12)
    assert np.allclose(r["b"], ro["b"], rtol=1e-10, atol=1e-12)
