"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (derived from the arithmetic; the method itself fixes E0 to 1e-10
relative in FP64 and 1e-6 in mixed precision):
  * FP64 H.v: every output is a sum of at most 1 + w_up + w_dn terms of size
    <= max(|U| * Ns, |t|) * max|x|; summed in a different order its error is
    below ~40 ulp of that scale, so max|y - y_ref| <= 1e-13 * max|y_ref| holds
    with a wide margin.
  * FP32 H.v (FP32 accumulation of FP32 inputs): per element
    |err| <= n u sum|terms| with u = 2^-24 and n <= 1 + w_up + w_dn; checked
    element-wise against that bound and norm-wise at 1e-5.
  * Lanczos: a_j, b_{j+1} agree with the oracle's from the same start vector
    while rounding has not yet been amplified (first 20 steps, 1e-12 relative;
    Sec. 5 reports this same check), and E0 within 1e-10 relative (FP64) or
    1e-6 (mixed).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workload

torch = pytest.importorskip("torch")
hb = pytest.importorskip("paper_1204_3425_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _build(p):
    return hb.hubbard_build(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)


def _oracle(p):
    return oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)


def _apply_gpu(h, x_np, precision):
    hb.hubbard_set_precision(h, precision)
    dt = torch.float64 if precision == hb.HUBBARD_FP64 else torch.float32
    x = torch.from_numpy(x_np).to(DEV, dt)
    y = torch.empty_like(x)
    hb.hubbard_apply(h, x, y)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _apply_gpu_ld(h, x_np, precision):
    """H x through hubbard_apply_ld on rows padded to ld_pref: the layout and
    kernels the Lanczos driver and the benchmark use."""
    hb.hubbard_set_precision(h, precision)
    dt = torch.float64 if precision == hb.HUBBARD_FP64 else torch.float32
    ld = hb.hubbard_info(h)["ld_pref"]
    xp = torch.zeros((h.dim_up, ld), dtype=dt, device=DEV)
    xp[:, :h.dim_dn] = torch.from_numpy(x_np).to(DEV, dt).view(h.dim_up, h.dim_dn)
    yp = torch.empty_like(xp)
    hb.hubbard_apply_ld(h, xp, ld, yp, ld)
    torch.cuda.synchronize()
    out = yp[:, :h.dim_dn].double().cpu().numpy().reshape(-1)
    del xp, yp
    return out


def _term_bound(p, info):
    return max(abs(p.U) * p.sites, abs(p.t)) * (1 + info["w_up"] + info["w_dn"])


APPLY_CASES = [
    workload.problem("ring8", 8, workload.ring(8), 4, 4, 1.0, 4.0),
    workload.problem("ring7_ragged", 7, workload.ring(7), 3, 2, 0.7, 2.5),
    workload.problem("torus3x4", 12, workload.torus(3, 4), 5, 6, 1.0, 8.0),
    workload.problem("ring10_U0", 10, workload.ring(10), 4, 5, 1.3, 0.0),
    workload.problem("ring10_t0", 10, workload.ring(10), 5, 5, 0.0, 3.0),
    workload.problem("dn_empty", 9, workload.ring(9), 4, 0, 1.0, 2.0),
    workload.problem("up_empty", 9, workload.ring(9), 0, 4, 1.0, 2.0),
    workload.problem("single_state", 5, workload.ring(5), 5, 0, 1.0, 2.0),
    workload.problem("chain11", 11, workload.chain(11), 5, 6, 1.0, 5.0),
    # dim_dn * 8 bytes > 160 KB: the down-spin rows do not fit in LDS
    workload.problem("ring18_wide_rows", 18, workload.ring(18), 1, 9, 1.0, 4.0),
    workload.problem("ring14", 14, workload.ring(14), 7, 7, 1.0, 4.0),
] + [
    # the 4x4 lattice with 8 electrons of one spin (1,544,400 states): down rows
    # of 12,870 elements as in the headline sector, and 12,870 up rows in the
    # headline sector's row blocks, with a full element-wise check
    workload.problem("sq4x4_2u8d", 16, workload.torus(4, 4), 2, 8, 1.0, 8.0),
    workload.problem("sq4x4_8u2d", 16, workload.torus(4, 4), 8, 2, 1.0, 8.0),
]


@pytest.mark.parametrize("p", APPLY_CASES, ids=[c.name for c in APPLY_CASES])
@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
def test_apply_matches_oracle(p, precision):
    _say("apply", p.name, "dim", p.dim, "precision", precision)
    h = _build(p)
    m = _oracle(p)
    x = workload.random_vector(p.dim, p.seed + 1)
    if precision == hb.HUBBARD_MIXED:
        x = x.astype(np.float32).astype(np.float64)
    ref = m.apply(x)
    got = _apply_gpu(h, x, precision)
    scale = max(1.0, np.abs(ref).max())
    if precision == hb.HUBBARD_FP64:
        assert np.abs(got - ref).max() <= 1e-13 * scale
    else:
        info = hb.hubbard_info(h)
        bound = (1 + info["w_up"] + info["w_dn"]) * 2.0**-24 * _term_bound(p, info) * np.abs(x).max()
        assert np.abs(got - ref).max() <= bound
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref) + 1e-30


PADDED_CASES = [
    # more than 1024 up configurations: several row blocks, hops inside and across blocks
    workload.problem("ring14", 14, workload.ring(14), 7, 7, 1.0, 4.0),
    workload.problem("torus3x4_t07", 12, workload.torus(3, 4), 6, 5, 0.7, 3.0),
    # every pair of 12 sites bonded: up rows of 36 hops (the two-line, 64-slot layout)
    workload.problem("complete12", 12, [(i, j) for i in range(12) for j in range(i + 1, 12)], 6, 2, 1.0, 2.0),
    # every pair of 17 sites bonded, 8 up: up rows of 72 hops, more than the line
    # layouts hold (the variable-width blocked pass)
    workload.problem("complete17_8u1d", 17, [(i, j) for i in range(17) for j in range(i + 1, 17)], 8, 1, 1.0, 3.0),
    workload.problem("chain13_ragged", 13, workload.chain(13), 7, 3, 1.0, 5.0),
    # down rows of 12,870 elements on the 4x4 lattice (the headline sector's
    # row-pass launch shape: one row per workgroup in FP64, a row pair in FP32) ...
    workload.problem("sq4x4_2u8d", 16, workload.torus(4, 4), 2, 8, 1.0, 8.0),
    workload.problem("sq4x4_1u8d_U0", 16, workload.torus(4, 4), 1, 8, 1.3, 0.0),
    # ... and 12,870 up rows in its 16 row blocks (the line pass of the headline sector)
    workload.problem("sq4x4_8u2d", 16, workload.torus(4, 4), 8, 2, 1.0, 8.0),
    workload.problem("sq4x4_8u1d_ragged", 16, workload.torus(4, 4), 8, 1, 0.8, 3.0),
]


@pytest.mark.parametrize("p", PADDED_CASES, ids=[c.name for c in PADDED_CASES])
@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
def test_apply_padded_rows_match_oracle(p, precision):
    _say("apply padded", p.name, "dim", p.dim, "precision", precision)
    h = _build(p)
    m = _oracle(p)
    x = workload.random_vector(p.dim, p.seed + 4)
    if precision == hb.HUBBARD_MIXED:
        x = x.astype(np.float32).astype(np.float64)
    ref = m.apply(x)
    got = _apply_gpu_ld(h, x, precision)
    scale = max(1.0, np.abs(ref).max())
    if precision == hb.HUBBARD_FP64:
        assert np.abs(got - ref).max() <= 1e-13 * scale
    else:
        info = hb.hubbard_info(h)
        bound = (1 + info["w_up"] + info["w_dn"]) * 2.0**-24 * _term_bound(p, info) * np.abs(x).max()
        assert np.abs(got - ref).max() <= bound


@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
def test_apply_4x4_full_vector(precision):
    """The 4x4 half-filled sector (dim 165,636,900) at full size, in the launch
    configuration the benchmark uses (rows padded to ld_pref): every output
    against the oracle's H.v (about 10 s on one host core), and the symmetry of
    H against the kernels for dense caller rows."""
    p = workload.square4x4()
    _say("apply 4x4 full vector, precision", precision)
    h = _build(p)
    m = _oracle(p)
    x = workload.random_vector(p.dim, p.seed + 2)
    if precision == hb.HUBBARD_MIXED:
        x = x.astype(np.float32).astype(np.float64)
    got = _apply_gpu_ld(h, x, precision)
    ref = m.apply(x)
    err = np.abs(got - ref)
    _say("4x4 max abs err %.3e (max |ref| %.3e)" % (err.max(), np.abs(ref).max()))
    if precision == hb.HUBBARD_FP64:
        assert err.max() <= 1e-13 * max(1.0, np.abs(ref).max())
    else:
        info = hb.hubbard_info(h)
        bound = (1 + info["w_up"] + info["w_dn"]) * 2.0**-24 * _term_bound(p, info) * np.abs(x).max()
        assert err.max() <= bound
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    del err, ref
    # symmetry of H at full size: <u, H v> == <H u, v>
    u = workload.random_vector(p.dim, p.seed + 3)
    if precision == hb.HUBBARD_MIXED:
        u = u.astype(np.float32).astype(np.float64)
    Hu = _apply_gpu(h, u, precision)  # dense rows: the caller's J-order layout
    lhs, rhs = float(u @ got), float(Hu @ x)
    tol = 1e-11 if precision == hb.HUBBARD_FP64 else 1e-4
    assert abs(lhs - rhs) <= tol * (np.abs(u).sum() + np.abs(x).sum())


def test_apply_ring16_full_vector():
    """The 16-site ring at half filling (dim 165,636,900, 16-hop rows: a
    different table structure from the 4x4 lattice at the same size), FP64 on
    padded rows, every output against the oracle's H.v."""
    p = workload.problem("ring16", 16, workload.ring(16), 8, 8, 1.0, 6.0)
    _say("apply ring16 full vector")
    h = _build(p)
    m = _oracle(p)
    x = workload.random_vector(p.dim, p.seed + 5)
    got = _apply_gpu_ld(h, x, hb.HUBBARD_FP64)
    ref = m.apply(x)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("pad", [0, 3, 64])
def test_apply_strided_rows_equal_dense(precision, pad):
    """hubbard_apply_ld on padded rows gives bitwise the dense result, and
    leaves the padding untouched."""
    p = workload.problem("torus3x4", 12, workload.torus(3, 4), 5, 6, 1.0, 8.0)
    h = _build(p)
    hb.hubbard_set_precision(h, precision)
    dt = torch.float64 if precision == hb.HUBBARD_FP64 else torch.float32
    info = hb.hubbard_info(h)
    ld = info["ld_pref"] + pad
    x = torch.from_numpy(workload.random_vector(p.dim, 5)).to(DEV, dt)
    y = torch.empty_like(x)
    hb.hubbard_apply(h, x, y)
    xp = torch.full((p.dim_up, ld), 7.0, dtype=dt, device=DEV)
    xp[:, :p.dim_dn] = x.view(p.dim_up, p.dim_dn)
    yp = torch.full((p.dim_up, ld), -3.0, dtype=dt, device=DEV)
    hb.hubbard_apply_ld(h, xp, ld, yp, ld)
    torch.cuda.synchronize()
    assert torch.equal(yp[:, :p.dim_dn].reshape(-1), y)
    assert bool((yp[:, p.dim_dn:] == -3.0).all())


def test_apply_rejects_overlap_and_bad_tensors():
    p = workload.ring8()
    h = _build(p)
    x = torch.zeros(p.dim * 2, dtype=torch.float64, device=DEV)
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_apply(h, x.data_ptr(), x.data_ptr() + 8 * 100)
    assert ei.value.code == hb.HUBBARD_EINVAL
    with pytest.raises(TypeError):
        hb.hubbard_apply(h, torch.zeros(p.dim, device=DEV), torch.zeros(p.dim, device=DEV))
    with pytest.raises(ValueError):
        hb.hubbard_apply(h, torch.zeros(p.dim + 1, dtype=torch.float64, device=DEV),
                         torch.zeros(p.dim, dtype=torch.float64, device=DEV))


def test_start_vector_bit_exact():
    """The device SplitMix64 start vector equals the oracle's bit for bit."""
    for seed, dim in [(0, 1000), (workload.BASE_SEED, 123457), (2**63 + 11, 4900)]:
        f = torch.empty(dim, dtype=torch.float64, device=DEV)
        hb.hubbard_start_raw(seed, dim, f)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), oracle.start_vector(seed, dim, normalise=False))


def _lanczos_gpu(h, p, precision, tol, max_iter, want_psi=False, start=None):
    psi = torch.empty(p.dim, dtype=torch.float64, device=DEV) if want_psi else None
    r = hb.hubbard_lanczos_ex(h, tol=tol, max_iter=max_iter, precision=precision, seed=p.seed, psi=psi,
                              start=start)
    torch.cuda.synchronize()
    if want_psi:
        r["psi"] = psi.cpu().numpy()
    return r


def test_lanczos_ring8_fp64_matches_oracle():
    p = workload.ring8()
    _say("lanczos ring8 fp64")
    h = _build(p)
    m = _oracle(p)
    ref = m.lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=300, want_psi=True)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 300, want_psi=True)
    assert got["E0"] == pytest.approx(ref["E0"], rel=1e-10)
    k = 20
    assert np.allclose(got["a"][:k], ref["a"][:k], rtol=1e-12, atol=1e-13)
    assert np.allclose(got["b"][:k], ref["b"][:k], rtol=1e-12, atol=1e-13)
    assert got["stop"] == "converged"
    assert abs(np.linalg.norm(got["psi"]) - 1) < 1e-12
    assert abs(got["psi"] @ ref["psi"]) > 1 - 1e-8
    assert got["residual"] < 1e-5 and got["residual"] == pytest.approx(
        np.linalg.norm(m.apply(got["psi"]) - got["E0"] * got["psi"]), rel=1e-6, abs=1e-12)
    assert got["rayleigh"] == pytest.approx(ref["E0"], rel=1e-11)


def test_lanczos_ring8_plain_entry_point():
    p = workload.ring8()
    h = _build(p)
    hb.hubbard_set_seed(h, p.seed)
    rc, e0 = hb.hubbard_lanczos(h, 1e-12, 300)
    assert rc == hb.HUBBARD_OK
    ref = _oracle(p).lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=300)["E0"]
    assert e0 == pytest.approx(ref, rel=1e-10)
    rc, _ = hb.hubbard_lanczos(h, 1e-14, 3)
    assert rc == hb.HUBBARD_ENOCONV


def test_lanczos_given_start_vector():
    p = workload.problem("torus2x4", 8, workload.torus(2, 4), 3, 4, 1.0, 6.0)
    h = _build(p)
    m = _oracle(p)
    f = workload.random_vector(p.dim, 77)
    f /= np.linalg.norm(f)
    ref = m.lanczos(f, tol=1e-12, max_iter=200)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 200, start=torch.from_numpy(f).to(DEV))
    assert np.allclose(got["a"][:15], ref["a"][:15], rtol=1e-12, atol=1e-13)
    assert got["E0"] == pytest.approx(ref["E0"], rel=1e-10)


def test_lanczos_ring14_against_golden():
    """14-site ring, FP64 and mixed, against the stored oracle run (same seed)."""
    g = json.load(open(os.path.join(GOLDEN, "oracle_ring14.json")))
    p = workload.ring14()
    assert g["problem"]["dim"] == p.dim and g["problem"]["seed"] == p.seed
    h = _build(p)
    _say("lanczos ring14 fp64")
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 400, want_psi=True)
    assert got["E0"] == pytest.approx(g["E0"], rel=1e-10)
    assert np.allclose(got["a"][:20], g["a"][:20], rtol=1e-12, atol=1e-13)
    assert np.allclose(got["b"][:20], g["b"][:20], rtol=1e-12, atol=1e-13)
    assert got["residual"] < 1e-4
    _say("lanczos ring14 mixed")
    mix = _lanczos_gpu(h, p, hb.HUBBARD_MIXED, 1e-10, 400, want_psi=True)
    assert mix["E0"] == pytest.approx(g["E0"], rel=1e-6)
    assert mix["rayleigh"] == pytest.approx(g["E0"], rel=1e-6)
    assert mix["residual"] < 1e-2


def test_lanczos_4x4_against_golden():
    path = os.path.join(GOLDEN, "oracle_square4x4.json")
    if not os.path.exists(path):
        pytest.skip("4x4 oracle run not stored")
    g = json.load(open(path))
    p = workload.square4x4()
    h = _build(p)
    n = g["max_iter"]
    _say("lanczos 4x4 fp64", n)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, -1.0, n)
    assert got["n_iter"] == g["n_iter"]
    # Each a_j, b_{j+1} is a dot product over dim = 1.66e8 terms; two summation
    # orders differ by about sqrt(dim) * eps ~ 1.4e-12 relative per step, and the
    # recurrence carries that forward, so the first 20 steps are compared at
    # 64 sqrt(dim) eps (= 9e-11) rather than the small-sector 1e-12.
    rtol = 64 * math.sqrt(p.dim) * np.finfo(np.float64).eps
    da = np.abs(got["a"][:20] - g["a"][:20]) / np.abs(np.asarray(g["a"][:20]))
    db = np.abs(got["b"][:20] - g["b"][:20]) / np.abs(np.asarray(g["b"][:20]))
    _say("4x4 first-20 max rel diff a %.2e b %.2e (tol %.2e)" % (da.max(), db.max(), rtol))
    assert da.max() <= rtol and db.max() <= rtol
    assert got["E0"] == pytest.approx(g["E0"], rel=1e-10)
    _say("lanczos 4x4 mixed", n)
    mix = _lanczos_gpu(h, p, hb.HUBBARD_MIXED, -1.0, n)
    assert mix["E0"] == pytest.approx(g["E0"], rel=1e-6)


def test_lanczos_large_sector_matches_oracle():
    """A 392,040-state sector: large enough for the fused step (the update
    q - a_j f_j formed inside the next H.v, b_{j+1} from the expanded norm),
    small enough for the oracle to follow with psi."""
    p = workload.problem("torus3x4_4u5d", 12, workload.torus(3, 4), 4, 5, 1.0, 6.0)
    h = _build(p)
    m = _oracle(p)
    _say("oracle lanczos", p.name, p.dim)
    ref = m.lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=300, want_psi=True)
    for prec in (hb.HUBBARD_FP64, hb.HUBBARD_MIXED):
        _say("lanczos", p.name, prec)
        got = _lanczos_gpu(h, p, prec, 1e-12 if prec == hb.HUBBARD_FP64 else 1e-9, 300, want_psi=True)
        if prec == hb.HUBBARD_FP64:
            assert got["E0"] == pytest.approx(ref["E0"], rel=1e-10)
            assert np.allclose(got["a"][:20], ref["a"][:20], rtol=1e-12, atol=1e-13)
            assert np.allclose(got["b"][:20], ref["b"][:20], rtol=1e-12, atol=1e-13)
            assert abs(got["psi"] @ ref["psi"]) > 1 - 1e-8
            assert got["rayleigh"] == pytest.approx(ref["E0"], rel=1e-11)
        else:
            assert got["E0"] == pytest.approx(ref["E0"], rel=1e-6)
            assert abs(got["psi"] @ ref["psi"]) > 1 - 1e-4
        assert got["residual"] == pytest.approx(
            np.linalg.norm(m.apply(got["psi"]) - got["E0"] * got["psi"]), rel=1e-6, abs=1e-12)


def test_lanczos_wide_up_rows():
    """Up rows of 36 hops (every pair of 12 sites bonded), 203,280 states: the
    fused step on the blocked pass for rows longer than one 32-slot line."""
    p = workload.problem("complete12_6u3d", 12, [(i, j) for i in range(12) for j in range(i + 1, 12)], 6, 3,
                         1.0, 2.0)
    h = _build(p)
    assert hb.hubbard_info(h)["w_up"] > 32
    ref = _oracle(p).lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=300)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 300)
    assert got["E0"] == pytest.approx(ref["E0"], rel=1e-10)
    assert np.allclose(got["a"][:20], ref["a"][:20], rtol=1e-12, atol=1e-13)


def test_lanczos_up_rows_over_64_hops():
    """Up rows of up to 72 hops (17 sites, each pair bonded with probability 0.9,
    seeded: 128 bonds; 8 up + 1 down, 413,270 states): the fused step on the
    variable-width blocked pass for 20 steps.  (The complete graph has so few
    distinct energies that its Krylov space ends after about ten steps.)"""
    g = np.random.default_rng(17)
    edges = [(i, j) for i in range(17) for j in range(i + 1, 17) if g.random() < 0.9]
    p = workload.problem("dense17_8u1d", 17, edges, 8, 1, 1.0, 3.0)
    h = _build(p)
    assert hb.hubbard_info(h)["w_up"] > 64
    ref = _oracle(p).lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-300, max_iter=20)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, -1.0, 20)
    assert np.allclose(got["a"], ref["a"], rtol=1e-12, atol=1e-12)
    assert np.allclose(got["b"], ref["b"], rtol=1e-10, atol=1e-12)


def test_lanczos_fused_step_decaying_b():
    """A fused-size sector (392,040 states) in the atomic limit (t = 0: H is
    diagonal with the levels U * D, D the double occupancy) from a start vector
    whose weight on each level falls by 1e4 per doubly occupied site: the
    Krylov vectors are dominated by successive levels and b_{j+1} / |q_j|
    falls to about 3.6e-5, where |q|^2 - 2 c q.f + c^2 |f|^2 loses most digits
    of b_{j+1} (about 1e-8 of it here).  Such steps take the explicit norm.
    Compared: a_1..a_4 and b_2..b_4.  b_5 is left out: it measures the weight
    of the highest level (D = 4) in f_4, and the start vector gives that level
    1e-16 of the amplitude of the lowest one: the size of the rounding errors
    every step of the recurrence adds to all levels, so b_5 is set by rounding
    on both sides (they differ by about 1e-5 of it)."""
    p = workload.problem("torus3x4_atomic_decay", 12, workload.torus(3, 4), 4, 5, 0.0, 4.0)
    h = _build(p)
    m = _oracle(p)
    D = np.rint(m.diagonal() / p.U).astype(int)
    f = workload.random_vector(p.dim, 3) * (10.0 ** (-4.0 * D))
    f /= np.linalg.norm(f)
    ref = m.lanczos(f, tol=-1.0, max_iter=4)
    qq = (np.asarray(ref["a"]) ** 2 + np.asarray(ref["b"]) ** 2) / np.asarray(ref["b"]) ** 2
    assert qq.max() > 1e8  # the regime the explicit norm is for
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, -1.0, 4, start=torch.from_numpy(f).to(DEV))
    _say("decaying b: max rel diff a %.2e b %.2e" % (
        np.max(np.abs(got["a"] - ref["a"]) / np.abs(ref["a"])), np.max(np.abs(got["b"] - ref["b"]) / ref["b"])))
    assert np.allclose(got["a"], ref["a"], rtol=1e-10, atol=0)
    assert np.allclose(got["b"][:3], ref["b"][:3], rtol=1e-10, atol=0)


def test_lanczos_large_sector_breakdown():
    """Atomic limit (t = 0) of a fused-size sector from a start vector in the
    span of two basis states: the Krylov space is that plane, the run stops
    with a breakdown after two steps, and E0 is the lower diagonal element."""
    p = workload.problem("torus3x4_atomic", 12, workload.torus(3, 4), 4, 5, 0.0, 4.0)
    h = _build(p)
    diag = _oracle(p).diagonal()
    J = 0
    K = int(np.flatnonzero(diag != diag[J])[0])
    f = np.zeros(p.dim)
    f[J] = f[K] = 1.0 / math.sqrt(2.0)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 50, want_psi=True, start=torch.from_numpy(f).to(DEV))
    assert got["stop"] == "breakdown" and got["n_iter"] == 2
    assert got["E0"] == pytest.approx(min(diag[J], diag[K]), rel=1e-12, abs=1e-12)
    assert got["residual"] < 1e-10


def test_lanczos_is_deterministic():
    p = workload.problem("torus3x4", 12, workload.torus(3, 4), 4, 5, 1.0, 6.0)
    h = _build(p)
    r1 = _lanczos_gpu(h, p, hb.HUBBARD_MIXED, -1.0, 60)
    r2 = _lanczos_gpu(h, p, hb.HUBBARD_MIXED, -1.0, 60)
    assert np.array_equal(r1["a"], r2["a"]) and np.array_equal(r1["b"], r2["b"])


@pytest.mark.parametrize("p", [
    workload.problem("one_state", 4, workload.ring(4), 4, 0, 1.0, 2.0),
    workload.problem("dimer", 2, [(0, 1)], 1, 1, 1.0, 4.0),
    workload.problem("tiny3", 3, workload.ring(3), 1, 1, 1.0, 1.0),
], ids=lambda p: p.name)
def test_lanczos_degenerate_sectors(p):
    """dim 1 (breakdown at once), the dimer closed form, a 9-state sector that
    exhausts its Krylov space."""
    h = _build(p)
    m = _oracle(p)
    ref = m.lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=50, want_psi=True)
    got = _lanczos_gpu(h, p, hb.HUBBARD_FP64, 1e-12, 50, want_psi=True)
    assert got["E0"] == pytest.approx(ref["E0"], rel=1e-10, abs=1e-12)
    assert got["n_iter"] == ref["n_iter"]
    assert got["residual"] < 1e-6
    if p.name == "dimer":
        assert got["E0"] == pytest.approx(2 - math.sqrt(4 + 4), rel=1e-12)


_ORACLE_E0 = {}


def _oracle_run(p):
    """Oracle Lanczos from the problem's seed, cached per problem."""
    if p not in _ORACLE_E0:
        _ORACLE_E0[p] = _oracle(p).lanczos(oracle.start_vector(p.seed, p.dim), tol=1e-12, max_iter=300)
    return _ORACLE_E0[p]


def _batch(handles, probs, precision, tol=1e-10, max_iter=300, psis=None):
    r = hb.hubbard_lanczos_batch(handles, tol=tol, max_iter=max_iter, precision=precision,
                                 seeds=[p.seed for p in probs], psis=psis, history=True)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("precision", [hb.HUBBARD_FP64, hb.HUBBARD_MIXED], ids=["fp64", "mixed"])
def test_batch_matches_oracle_and_solo(precision):
    """Batched solves (shared launches) against the oracle and against the
    single-instance path."""
    probs = workload.batch64(8)
    hs = [_build(p) for p in probs]
    _say("batch of", len(probs), "precision", precision)
    # the oracle runs stop at an energy change of 1e-12; the FP64 runs use the same test
    tol = 1e-12 if precision == hb.HUBBARD_FP64 else 1e-10
    got = _batch(hs, probs, precision, tol=tol)
    rel = 1e-10 if precision == hb.HUBBARD_FP64 else 1e-6
    for g, h, p in zip(got, hs, probs):
        ref = _oracle_run(p)
        assert g["E0"] == pytest.approx(ref["E0"], rel=rel), p.name
        assert g["stop"] in ("converged", "breakdown", "exhausted"), p.name
        assert 0 <= g["err_est"] < 1e-3, p.name
        solo = _lanczos_gpu(h, p, precision, tol, 300)
        assert g["E0"] == pytest.approx(solo["E0"], rel=rel), p.name
        if precision == hb.HUBBARD_FP64:
            assert np.allclose(g["a"][:10], solo["a"][:10], rtol=1e-12, atol=1e-13)


def test_batch_result_independent_of_mix():
    """An instance gives bitwise the same a_j, b_{j+1}, E0 alone and inside a
    batch of 64 (per-instance work items and fixed-order reductions)."""
    probs = workload.batch64(64)
    hs = [_build(p) for p in probs]
    mix = _batch(hs, probs, hb.HUBBARD_MIXED)
    for k in (0, 17, 63):
        alone = _batch([hs[k]], [probs[k]], hb.HUBBARD_MIXED)[0]
        assert alone["n_iter"] == mix[k]["n_iter"]
        assert np.array_equal(alone["a"], mix[k]["a"]) and np.array_equal(alone["b"], mix[k]["b"])
        assert alone["E0"] == mix[k]["E0"]


def test_batch_stop_rules_match_single_instance():
    """The batched stop tests (computed on the device) against the single-
    instance driver: a 1-state sector (breakdown at once), the dimer, a 9-state
    sector that exhausts its Krylov space, a fixed step count (tol < 0) and an
    iteration cap, in one batch."""
    probs = [workload.problem("one_state", 4, workload.ring(4), 4, 0, 1.0, 2.0),
             workload.problem("dimer", 2, [(0, 1)], 1, 1, 1.0, 4.0),
             workload.problem("tiny3", 3, workload.ring(3), 1, 1, 1.0, 1.0),
             workload.ring8(), workload.ring8()]
    hs = [_build(p) for p in probs]
    opts = [(1e-12, 50), (1e-12, 50), (1e-12, 50), (-1.0, 37), (1e-14, 12)]
    got = []
    for (tol, mi), h, p in zip(opts, hs, probs):
        got.append(hb.hubbard_lanczos_batch([h], tol=tol, max_iter=mi, precision=hb.HUBBARD_FP64,
                                            seeds=[p.seed], history=True)[0])
    mixed = [hb.hubbard_lanczos_batch(hs, tol=opts[0][0], max_iter=50, precision=hb.HUBBARD_FP64,
                                      seeds=[p.seed for p in probs], history=True)]
    for (tol, mi), h, p, g in zip(opts, hs, probs, got):
        solo = _lanczos_gpu(h, p, hb.HUBBARD_FP64, tol, mi)
        assert g["stop"] == solo["stop"], p.name
        assert g["n_iter"] == solo["n_iter"], p.name
        assert g["E0"] == pytest.approx(solo["E0"], rel=1e-12, abs=1e-13), p.name
        assert np.allclose(g["a"], solo["a"], rtol=1e-12, atol=1e-13)
    assert got[3]["stop"] == "max_iter" and got[3]["n_iter"] == 37
    assert got[4]["stop"] == "max_iter" and got[4]["status"] == hb.HUBBARD_ENOCONV
    # the first three again inside one batch with the others
    for k in range(3):
        assert mixed[0][k]["E0"] == got[k]["E0"] and mixed[0][k]["n_iter"] == got[k]["n_iter"]


def test_batch_with_psi_requests_and_large_rows():
    """Solves that ask for psi, or whose rows exceed the batched kernels' LDS,
    run on the single-instance path inside the same call."""
    probs = workload.batch64(3) + [workload.problem("wide", 18, workload.ring(18), 1, 9, 1.0, 3.0, seed=7)]
    hs = [_build(p) for p in probs]
    psis = [None, torch.empty(probs[1].dim, dtype=torch.float64, device=DEV), None, None]
    got = _batch(hs, probs, hb.HUBBARD_FP64, tol=1e-12, psis=psis)
    for g, p in zip(got, probs):
        assert g["E0"] == pytest.approx(_oracle_run(p)["E0"], rel=1e-10), p.name
    assert got[1]["residual"] >= 0 and got[0]["residual"] == -1
