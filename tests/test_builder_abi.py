"""Host-side checks of the GPU library (CPU only): the C ABI loads and exports
every declared symbol, the basis and ELL hopping tables are bit-exact against
the oracle, and argument validation returns the documented codes."""
import ctypes
import math
import re

import numpy as np
import pytest

import oracle
import workload
from conftest import golden_rows

hb = pytest.importorskip("paper_1204_3425_amd")


def ell_pack_column_major(rows, width):
    """Test-side ELL packer (Sec. 4.2, Fig. ELL): each row's (col, value) pairs in
    order, padded to `width` with (pad_col, pad_val), flattened column-major."""
    n = len(rows)
    cols = np.zeros((width, n), dtype=np.int64)
    vals = np.zeros((width, n), dtype=np.float64)
    for r, row in enumerate(rows):
        for k, (c, v) in enumerate(row):
            cols[k, r] = c
            vals[k, r] = v
    return cols.reshape(-1), vals.reshape(-1)


def test_ell_packer_reproduces_figure():
    """The test packer gives Fig. ELL's column-major data and index vectors."""
    lines = golden_rows("ell_example.txt")
    i_m, i_d, i_x = [k for k, ln in enumerate(lines) if ln[0] in ("matrix", "data", "indices")]
    A = np.array([[float(v) for v in ln] for ln in lines[i_m + 1:i_d]])
    rows = [[(c, A[r, c]) for c in range(A.shape[1]) if A[r, c] != 0] for r in range(A.shape[0])]
    w = max(len(r) for r in rows)
    cols, vals = ell_pack_column_major(rows, w)
    want_d = lines[i_d + 1]
    want_i = lines[i_x + 1]
    assert len(want_d) == len(vals) == len(want_i)
    for k in range(len(vals)):
        if want_d[k] == "*":
            assert vals[k] == 0 and cols[k] == 0  # padding set to zero
        else:
            assert vals[k] == float(want_d[k]) and cols[k] == int(want_i[k])


def test_every_declared_symbol_is_exported():
    text = open(hb.HEADER_PATH).read()
    names = sorted(set(re.findall(r"\b(hubbard_[a-z_0-9]+)\s*\(", text)))
    assert "hubbard_build" in names and "hubbard_lanczos" in names and "hubbard_apply" in names
    lib = ctypes.CDLL(hb.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


CASES = [
    (4, workload.ring(4), 2, 3),
    (6, workload.torus(2, 3), 3, 2),
    (8, workload.ring(8), 4, 4),
    (10, workload.ring(10), 3, 5),
    (12, workload.torus(3, 4), 6, 5),
    (12, workload.torus(4, 3), 4, 8),
    (14, workload.ring(14), 7, 7),
    (16, workload.torus(4, 4), 8, 8),
    (16, workload.torus(4, 4), 5, 3),
    (9, workload.chain(9), 0, 9),
]


@pytest.mark.parametrize("ns,edges,nu,nd", CASES)
def test_basis_and_tables_bit_exact(ns, edges, nu, nd):
    """Basis words and signed ELL tables equal the oracle's (Sec. 2.1, Sec. 4.2)."""
    h = hb.hubbard_build(ns, edges, nu, nd, 1.0, 4.0)
    m = oracle.Model(ns, edges, nu, nd, 1.0, 4.0)
    info = hb.hubbard_info(h)
    assert info["dim"] == m.dim == math.comb(ns, nu) * math.comb(ns, nd)
    for spin in (0, 1):
        states, rs, col, val = m.table(spin)
        assert np.array_equal(hb.hubbard_export_basis(h, spin), states)
        d = len(states)
        width = int(np.diff(rs).max()) if d else 0
        assert info["w_up" if spin == 0 else "w_dn"] == width
        assert info["nnz_up" if spin == 0 else "nnz_dn"] == len(col)
        # oracle values are -t * sgn with t = 1
        rows = [[(int(col[k]), -val[k]) for k in range(rs[r], rs[r + 1])] for r in range(d)]
        want_col, want_sgn = ell_pack_column_major(rows, width)
        got_col, got_sgn = hb.hubbard_export_table(h, spin)
        assert np.array_equal(got_col, want_col)
        assert np.array_equal(got_sgn.astype(np.float64), want_sgn)


def test_table1_through_export():
    """Sec. 2.1, Table 1, read through the library's exported basis."""
    h = hb.hubbard_build(4, workload.ring(4), 2, 3, 1.0, 0.0)
    up, dn = list(hb.hubbard_export_basis(h, 0)), list(hb.hubbard_export_basis(h, 1))
    for u, d, iu, idn, J in golden_rows("table1_labels.txt"):
        assert up.index(int(u, 2)) == int(iu) and dn.index(int(d, 2)) == int(idn)
        assert int(iu) * h.dim_dn + int(idn) == int(J)


@pytest.mark.parametrize("ns,edges,n,width", [(8, workload.ring(8), 4, 8), (14, workload.ring(14), 7, 14),
                                              (16, workload.torus(4, 4), 8, 32)])
def test_widths_and_nnz_closed_form(ns, edges, n, width):
    info = hb.hubbard_info(hb.hubbard_build(ns, edges, n, n, 1.0, 1.0))
    assert info["w_up"] == info["w_dn"] == width
    assert info["nnz_up"] == 2 * len(edges) * math.comb(ns - 2, n - 1)


@pytest.mark.parametrize("args", [
    (0, [], 0, 0), (33, [], 1, 1), (4, [(0, 4)], 1, 1), (4, [(1, 1)], 1, 1), (4, [(0, 1), (1, 0)], 1, 1),
    (4, [(0, 1)], 5, 1), (4, [(0, 1)], 1, -1), (4, [(-1, 2)], 1, 1)])
def test_invalid_build_arguments(args):
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build(*args, t=1.0, U=1.0)
    assert ei.value.code == hb.HUBBARD_EINVAL


@pytest.mark.parametrize("t,U", [(float("nan"), 1.0), (1.0, float("inf"))])
def test_non_finite_parameters(t, U):
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build(4, workload.ring(4), 2, 2, t, U)
    assert ei.value.code == hb.HUBBARD_EINVAL


def test_range_error():
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build(32, workload.ring(32), 16, 16, 1.0, 1.0)
    assert ei.value.code == hb.HUBBARD_ERANGE


def test_null_arguments_rejected():
    lib = ctypes.CDLL(hb.LIB_PATH)
    lib.hubbard_build.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    assert lib.hubbard_build(4, None, 0, 1, 1, 1.0, 1.0, None) == hb.HUBBARD_EINVAL
    assert lib.hubbard_build(4, None, 2, 1, 1, 1.0, 1.0, None) == hb.HUBBARD_EINVAL
    lib.hubbard_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.hubbard_info(None, None) == hb.HUBBARD_EINVAL
    lib.hubbard_free.argtypes = [ctypes.c_void_p]
    assert lib.hubbard_free(None) == hb.HUBBARD_OK


def test_strerror_and_last_error():
    assert hb.hubbard_strerror(hb.HUBBARD_EINVAL) == "invalid argument"
    with pytest.raises(hb.HubbardError):
        hb.hubbard_build(4, [(0, 0)], 1, 1)
    assert "distinct" in hb.hubbard_last_error()


def test_precision_and_seed_setters():
    h = hb.hubbard_build(4, workload.ring(4), 2, 2)
    hb.hubbard_set_precision(h, hb.HUBBARD_MIXED)
    hb.hubbard_set_seed(h, 5)
    with pytest.raises(hb.HubbardError):
        hb.hubbard_set_precision(h, 7)


def test_apply_ld_validates_strides_before_touching_the_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("uses made-up device addresses; run only where no GPU is present")
    h = hb.hubbard_build(6, workload.ring(6), 3, 3, 1.0, 2.0)
    lib = ctypes.CDLL(hb.LIB_PATH)
    lib.hubbard_apply_ld.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
    # stride shorter than a row
    assert lib.hubbard_apply_ld(h.ptr, 4096, h.dim_dn - 1, 1 << 30, h.dim_dn) == hb.HUBBARD_EINVAL
    # overlapping rows of x and y
    assert lib.hubbard_apply_ld(h.ptr, 4096, h.dim_dn, 4096 + 8, h.dim_dn) == hb.HUBBARD_EINVAL
    info = hb.hubbard_info(h)
    assert info["ld_pref"] >= h.dim_dn and info["ld_pref"] % 64 == 0


def test_admission_plan_first_fit():
    """The server's admission rule: first fit in arrival order under the budget
    and the free slots."""
    assert hb.hubbard_admission_plan([10, 20, 30], 100, 0, 8) == [1, 1, 1]
    assert hb.hubbard_admission_plan([10, 20, 30], 100, 50, 8) == [1, 1, 0]
    # a request that does not fit does not block smaller ones behind it
    assert hb.hubbard_admission_plan([60, 30, 10], 100, 50, 8) == [0, 1, 1]
    assert hb.hubbard_admission_plan([10, 10, 10], 100, 0, 2) == [1, 1, 0]
    assert hb.hubbard_admission_plan([10], 100, 200, 4) == [0]
    assert hb.hubbard_admission_plan([], 100, 0, 4) == []
    # never over the budget, whatever the mix
    rng = np.random.default_rng(1)
    for _ in range(200):
        fp = rng.integers(1, 50, size=12)
        used = int(rng.integers(0, 100))
        take = hb.hubbard_admission_plan(fp, 100, used, int(rng.integers(0, 6)))
        assert used + sum(f for f, t in zip(fp, take) if t) <= max(100, used)


def test_lowest_states_validates_before_touching_the_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("checks the no-device return code; run only where no GPU is present")
    h = hb.hubbard_build(2, [(0, 1)], 1, 1, 1.0, 2.0)  # dim 4
    lib = ctypes.CDLL(hb.LIB_PATH)
    lib.hubbard_lowest_states.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(hb.hubbard_opts),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    o = hb.hubbard_opts()
    o.tol, o.max_iter, o.precision, o.seed = 1e-12, 50, hb.HUBBARD_FP64, 1
    E = np.zeros(17)
    for k in (0, -1, 5, 17):  # out of 1..16 or above dim = 4
        assert lib.hubbard_lowest_states(h.ptr, k, ctypes.byref(o), E.ctypes.data, None, None) == hb.HUBBARD_EINVAL
    assert lib.hubbard_lowest_states(h.ptr, 2, None, E.ctypes.data, None, None) == hb.HUBBARD_EINVAL
    assert lib.hubbard_lowest_states(h.ptr, 2, ctypes.byref(o), None, None, None) == hb.HUBBARD_EINVAL
    o.psi = 4096  # opts.psi is not how the vectors are returned
    assert lib.hubbard_lowest_states(h.ptr, 2, ctypes.byref(o), E.ctypes.data, None, None) == hb.HUBBARD_EINVAL
    o.psi = None
    o.max_iter = 0
    assert lib.hubbard_lowest_states(h.ptr, 2, ctypes.byref(o), E.ctypes.data, None, None) == hb.HUBBARD_EINVAL
    o.max_iter = 50
    # valid arguments reach the device check
    assert lib.hubbard_lowest_states(h.ptr, 2, ctypes.byref(o), E.ctypes.data, None, None) == hb.HUBBARD_EDEVICE


def test_observables_validates_before_touching_the_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("checks the no-device return code; run only where no GPU is present")
    h = hb.hubbard_build(4, workload.ring(4), 2, 2, 1.0, 2.0)
    lib = ctypes.CDLL(hb.LIB_PATH)
    lib.hubbard_observables.argtypes = [ctypes.c_void_p] * 5
    assert lib.hubbard_observables(h.ptr, None, None, None, None) == hb.HUBBARD_EINVAL
    assert lib.hubbard_observables(None, 4096, None, None, None) == hb.HUBBARD_EINVAL
    assert lib.hubbard_observables(h.ptr, 4096, None, None, None) == hb.HUBBARD_EDEVICE


def test_build_bonds_tables_and_validation():
    """Per-bond amplitudes change only the values, not the table structure; all
    amplitudes equal give the one-amplitude handle; bad amplitude lists fail
    before anything is built."""
    edges = workload.torus(2, 3)
    amps = np.linspace(0.5, 1.5, len(edges))
    hg = hb.hubbard_build_bonds(6, edges, amps, 3, 2, 2.0)
    hu = hb.hubbard_build(6, edges, 3, 2, 1.0, 2.0)
    for spin in (0, 1):
        cg, sg = hb.hubbard_export_table(hg, spin)
        cu, su = hb.hubbard_export_table(hu, spin)
        assert np.array_equal(cg, cu) and np.array_equal(sg, su)
    assert math.isnan(hb.hubbard_info(hg)["t"])
    h1 = hb.hubbard_build_bonds(6, edges, [0.8] * len(edges), 3, 2, 2.0)
    assert hb.hubbard_info(h1)["t"] == 0.8
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build_bonds(6, edges, [1.0, float("nan")] + [1.0] * (len(edges) - 2), 3, 2, 2.0)
    assert ei.value.code == hb.HUBBARD_EINVAL
    # 136 bonds of a complete graph on 17 sites with 136 distinct amplitudes: above the 127 classes
    full = [(i, j) for i in range(17) for j in range(i + 1, 17)]
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build_bonds(17, full, np.arange(1, len(full) + 1, dtype=float), 1, 1, 0.0)
    assert ei.value.code == hb.HUBBARD_EINVAL
    # a spin dimension of 2^24 or more cannot hold the class bits (C(28,14) > 2^24)
    with pytest.raises(hb.HubbardError) as ei:
        hb.hubbard_build_bonds(28, workload.ring(28), np.linspace(1, 2, 28), 14, 1, 0.0)
    assert ei.value.code == hb.HUBBARD_ERANGE
    with pytest.raises(ValueError):
        hb.hubbard_build_bonds(6, edges, [1.0], 3, 2, 2.0)


def test_basis_limit_setter():
    h = hb.hubbard_build(4, workload.ring(4), 2, 2, 1.0, 2.0)
    hb.hubbard_set_basis_limit(h, 0)
    hb.hubbard_set_basis_limit(h, 2 ** 40)
    lib = ctypes.CDLL(hb.LIB_PATH)
    lib.hubbard_set_basis_limit.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    assert lib.hubbard_set_basis_limit(None, 0) == hb.HUBBARD_EINVAL
