"""GPU parity of the site observables (hubbard_observables) against the oracle.

Both sides get the same FP64 vector, so they differ only in the order of the
FP64 sums of non-negative terms psi_J^2 * (0 or 1): every sum is at most
<n> <= 1 (densities) or <= N_up N_dn (the double occupancy summed over sites),
and a sum of dim positive terms in any order is within dim * eps of it, far
below the 1e-12 (absolute) the test allows except beyond ~4.5e3 terms, where the
bound used is 1e-15 * dim (blocked sums do much better than that).
Full size: the 4x4 ground state against the oracle on the same vector, and the
double occupancy against dE0/dU from the GPU's own solves at U +- 1e-3
(Hellmann-Feynman; central difference error ~ 1e-7).
"""
import math

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


def _compare(h, m, v_np, tol):
    v = torch.from_numpy(v_np).to(DEV)
    g = hb.hubbard_observables(h, v)
    o = m.observables(v_np)
    assert np.abs(g["dens"] - o["dens"]).max() <= tol
    assert np.abs(g["corr"] - o["corr"]).max() <= tol
    assert abs(g["docc"] - o["docc"]) <= tol * max(1.0, m.n_up * m.n_dn)
    return g, o


CASES = [
    # name, sites, edges, n_up, n_dn
    ("dimer_1u1d", 2, [(0, 1)], 1, 1),
    ("ring8_4u4d", 8, workload.ring(8), 4, 4),
    ("ring8_0u3d", 8, workload.ring(8), 0, 3),  # one up row
    # 4,368 down configurations: two 4,096-wide tiles, the second ragged
    ("torus4x4_2u5d", 16, workload.torus(4, 4), 2, 5),
    # more than 16 sites: the 32-site variant of the kernel
    ("ring20_1u2d", 20, workload.ring(20), 1, 2),
    ("ring24_1u2d", 24, workload.ring(24), 1, 2),
]


@pytest.mark.parametrize("name,sites,edges,nu,nd", CASES, ids=[c[0] for c in CASES])
def test_observables_random_vector(name, sites, edges, nu, nd):
    """A seeded non-normalised vector (the observables divide by <psi|psi>)."""
    _say("observables", name)
    h = hb.hubbard_build(sites, edges, nu, nd, 1.0, 2.0)
    m = oracle.Model(sites, edges, nu, nd, 1.0, 2.0)
    v = np.random.default_rng(workload.BASE_SEED).uniform(-1, 1, m.dim) * 3.0
    _compare(h, m, v, max(1e-12, 1e-15 * m.dim))


def test_observables_ground_state_ring8():
    p = workload.ring8()
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    psi = torch.zeros(h.dim, dtype=torch.float64, device=DEV)
    hb.hubbard_lanczos_ex(h, tol=1e-13, max_iter=400, precision=hb.HUBBARD_FP64, seed=p.seed, psi=psi)
    g, _ = _compare(h, m, psi.cpu().numpy(), 1e-12)
    # a translation-invariant ring: every site holds N_sigma / Ns
    assert np.allclose(g["dens"], 0.5, atol=1e-9)


def test_observables_zero_vector_rejected():
    h = hb.hubbard_build(4, workload.ring(4), 2, 2, 1.0, 2.0)
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_observables(h, torch.zeros(h.dim, dtype=torch.float64, device=DEV))
    assert ei.value.code == hb.HUBBARD_EINVAL


def test_observables_square4x4_full_size():
    """The 4x4 ground state (dim 165.6M): every observable against the oracle on
    the same vector, and D against dE0/dU."""
    p = workload.square4x4()
    _say("observables", p.name)
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    psi = torch.zeros(h.dim, dtype=torch.float64, device=DEV)
    r = hb.hubbard_lanczos_ex(h, tol=1e-12, max_iter=400, precision=hb.HUBBARD_FP64, seed=p.seed, psi=psi)
    g = hb.hubbard_observables(h, psi)
    _say("E0", r["E0"], "D", g["docc"])
    d = 1e-3
    e = []
    for s in (-1, 1):
        hs = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U + s * d)
        e.append(hb.hubbard_lanczos_ex(hs, tol=1e-13, max_iter=400, precision=hb.HUBBARD_FP64, seed=p.seed)["E0"])
        del hs
    fd = (e[1] - e[0]) / (2 * d)
    _say("dE0/dU", fd)
    assert g["docc"] == pytest.approx(fd, abs=1e-5)
    # E0 = <H_hop> + U D: the interaction part of the Rayleigh quotient is U D
    assert 0.0 < g["docc"] < 16 * 0.25
    v = psi.cpu().numpy()
    del psi
    torch.cuda.empty_cache()
    m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    o = m.observables(v)
    tol = 1e-15 * math.sqrt(h.dim) * 10
    assert np.abs(g["dens"] - o["dens"]).max() <= tol
    assert np.abs(g["corr"] - o["corr"]).max() <= tol
    assert abs(g["docc"] - o["docc"]) <= 16 * tol
