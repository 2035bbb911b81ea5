"""The allocation-free observables entry point (hubbard_observables_noalloc)
against hubbard_observables through the C ABI, on two calls in a row (the
second on a smaller sector, so the static scratch holds the first call's
values when the second starts), for lattices of at most 16 sites (same
workgroup grid: bitwise equal) and of more (fewer accumulating workgroups:
equal within the FP64 rounding of sums of non-negative terms, at most
dim * eps relative)."""
import numpy as np
import pytest

import workload

torch = pytest.importorskip("torch")
hb = pytest.importorskip("paper_1204_3425_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _both(sites, edges, nu, nd, seed):
    h = hb.hubbard_build(sites, edges, nu, nd, 1.0, 4.0)
    v = torch.from_numpy(workload.random_vector(h.dim, seed)).to(DEV)
    a = hb.hubbard_observables_noalloc(h, v)
    b = hb.hubbard_observables(h, v)
    torch.cuda.synchronize()
    print("noalloc", sites, nu, nd, "dim", h.dim, "docc", a["docc"], b["docc"], flush=True)
    return a, b, h.dim


@pytest.mark.parametrize("calls", [
    # at most 16 sites: a 1,019,200-state 4x4 sector, then the 4,900-state ring
    [(16, workload.torus(4, 4), 3, 4, 5), (8, workload.ring(8), 4, 4, 6)],
    # more than 16 sites: the 32-site accumulation on a capped grid, twice
    [(20, workload.ring(20), 2, 2, 7), (18, workload.ring(18), 1, 2, 8)],
], ids=["sites16", "sites20"])
def test_noalloc_matches_observables(calls):
    for sites, edges, nu, nd, seed in calls:
        a, b, dim = _both(sites, edges, nu, nd, seed)
        if sites <= 16:
            assert np.array_equal(a["dens"], b["dens"]) and np.array_equal(a["corr"], b["corr"])
            assert a["docc"] == b["docc"]
        else:
            tol = max(1e-14, 4.0 * dim * np.finfo(float).eps)
            assert np.allclose(a["dens"], b["dens"], rtol=tol, atol=0)
            assert np.allclose(a["corr"], b["corr"], rtol=tol, atol=1e-300)
            assert a["docc"] == pytest.approx(b["docc"], rel=tol)
        # the densities sum to the electron counts
        assert a["dens"][0].sum() == pytest.approx(nu, rel=1e-12)
        assert a["dens"][1].sum() == pytest.approx(nd, rel=1e-12)
