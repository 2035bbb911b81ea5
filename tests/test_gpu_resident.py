"""The resident Lanczos basis for psi (hubbard_set_basis_limit): psi combined
from the kept vectors against psi accumulated by the replayed recurrence.

Both sum y_j f_j over the same vectors in the same order (the combination may
contract the multiply-add differently), so they agree to a few ulp of max|psi|:
1e-12 here.  E0 and the Lanczos coefficients do not depend on how psi is made
and are compared exactly, the residuals to 1e-10.
"""
import numpy as np
import pytest

import workload

torch = pytest.importorskip("torch")
hb = pytest.importorskip("paper_1204_3425_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _solve(h, precision, limit, tol=1e-12):
    hb.hubbard_set_basis_limit(h, limit)
    psi = torch.zeros(h.dim, dtype=torch.float64, device=DEV)
    r = hb.hubbard_lanczos_ex(h, tol=tol, max_iter=400, precision=precision, seed=workload.BASE_SEED, psi=psi)
    torch.cuda.synchronize()
    return r, psi


@pytest.mark.parametrize("which,precision", [("ring14", hb.HUBBARD_FP64), ("ring14", hb.HUBBARD_MIXED),
                                             ("ring8", hb.HUBBARD_FP64), ("ring8", hb.HUBBARD_MIXED)],
                         ids=["ring14-fp64-fused", "ring14-mixed-fused", "ring8-fp64", "ring8-mixed"])
def test_resident_psi_matches_replay(which, precision):
    p = workload.ring14() if which == "ring14" else workload.ring8()
    _say("resident vs replay", p.name, precision)
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    tol = 1e-12 if precision == hb.HUBBARD_FP64 else 1e-10
    r1, psi1 = _solve(h, precision, 2 ** 62, tol)
    r0, psi0 = _solve(h, precision, 0, tol)
    assert r1["psi_resident"] == 1 and r0["psi_resident"] == 0
    assert r1["E0"] == r0["E0"] and np.array_equal(r1["a"], r0["a"])
    assert float((psi1 - psi0).abs().max()) <= 1e-12
    assert r1["residual"] == pytest.approx(r0["residual"], rel=1e-6, abs=1e-10)


def test_basis_limit_reached_mid_run_falls_back():
    """A limit of five vectors: the run needs more, frees the slots and replays."""
    p = workload.ring8()
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    ld = hb.hubbard_info(h)["ld_pref"]
    r5, psi5 = _solve(h, hb.HUBBARD_FP64, 5 * h.dim_up * ld * 8)
    r1, psi1 = _solve(h, hb.HUBBARD_FP64, 2 ** 62)
    assert r5["n_iter"] > 5 and r5["psi_resident"] == 0 and r1["psi_resident"] == 1
    assert float((psi1 - psi5).abs().max()) <= 1e-12


def test_fused_run_leaves_slots_mid_run():
    """The 14-site ring takes the fused step with its vectors formed in their
    slots; a limit of one chunk (32 vectors) runs out at step 32 of 87, where the
    two live vectors move to the work vectors and psi comes from the replay.
    The recurrence is the same arithmetic either way: coefficients bitwise."""
    p = workload.ring14()
    _say("slots left mid-run", p.name)
    h = hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    ld = hb.hubbard_info(h)["ld_pref"]
    r32, psi32 = _solve(h, hb.HUBBARD_FP64, 32 * h.dim_up * ld * 8)
    r1, psi1 = _solve(h, hb.HUBBARD_FP64, 2 ** 62)
    assert r32["n_iter"] > 32 and r32["psi_resident"] == 0 and r1["psi_resident"] == 1
    assert r32["E0"] == r1["E0"] and np.array_equal(r32["a"], r1["a"]) and np.array_equal(r32["b"], r1["b"])
    assert float((psi1 - psi32).abs().max()) <= 1e-12


def test_lowest_states_resident_and_replayed():
    h = hb.hubbard_build(8, workload.ring(8), 3, 3, 1.0, 4.0)
    out = []
    for limit in (2 ** 62, 0):
        hb.hubbard_set_basis_limit(h, limit)
        psi = torch.zeros((3, h.dim), dtype=torch.float64, device=DEV)
        E, res = hb.hubbard_lowest_states(h, 3, tol=1e-14, max_iter=600, precision=hb.HUBBARD_FP64, psi=psi)
        assert all(r["psi_resident"] == (1 if limit else 0) for r in res)
        out.append((E, psi.cpu().numpy()))
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-12
    # the two ways of forming psi_0 differ in rounding, which the deflated runs of
    # the upper states see: they may stop a step apart, so their vectors agree to
    # about the residual (~4e-7 at tol 1e-14 here)
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-5
