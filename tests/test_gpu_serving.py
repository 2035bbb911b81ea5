"""GPU tests of the continuous-batching server (requests of uneven sector
sizes sharing the device) against the oracle and against the same request run
alone."""
import time

import numpy as np
import pytest

import oracle
import workload

torch = pytest.importorskip("torch")
hb = pytest.importorskip("paper_1204_3425_amd")

pytestmark = pytest.mark.gpu

_REF = {}


def _oracle_e0(p):
    if p not in _REF:
        m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
        _REF[p] = m.lanczos(oracle.start_vector(p.seed, m.dim), tol=1e-12, max_iter=300)["E0"]
    return _REF[p]


def _submit(srv, p, precision=hb.HUBBARD_MIXED, tag=0, tol=1e-10):
    return hb.hubbard_server_submit(srv, p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U, tol=tol, max_iter=300,
                                    precision=precision, seed=p.seed, tag=tag)


def _collect(srv, n, timeout_s=240.0):
    out = {}
    t0 = time.time()
    while len(out) < n:
        assert time.time() - t0 < timeout_s, "server did not complete %d requests in time" % n
        for c in hb.hubbard_server_poll(srv, cap=64, timeout_us=200000):
            out[c["id"]] = c
    return out


def test_server_results_budget_and_continuous_admission():
    probs = workload.batch64(16)
    budget = 48 << 20  # room for a few of these sectors at a time
    srv = hb.hubbard_server_create(budget, 6)
    print("server: submitting", len(probs), "requests", flush=True)
    ids = {}
    for i, p in enumerate(probs):
        ids[_submit(srv, p, tag=i)] = p
    big = workload.square4x4()
    big_id = _submit(srv, big, precision=hb.HUBBARD_FP64)  # needs > 2.6 GB: can never fit
    res = _collect(srv, len(ids) + 1)
    st = hb.hubbard_server_stats(srv)
    hb.hubbard_server_destroy(srv)
    assert res[big_id]["status"] == hb.HUBBARD_ENOMEM
    for rid, p in ids.items():
        c = res[rid]
        assert c["status"] == hb.HUBBARD_OK, (p.name, c["status"])
        assert c["E0"] == pytest.approx(_oracle_e0(p), rel=1e-6), p.name
        assert c["t_submit"] <= c["t_admit"] <= c["t_start"] <= c["t_done"]
    assert st["peak_reserved"] <= st["budget"]
    assert st["completed"] == len(ids) + 1 and st["rejected"] == 1
    assert st["max_active_batch"] >= 2
    done = [res[r] for r in ids]
    first_done = min(c["t_done"] for c in done)
    # requests waited for memory or a slot and were admitted as earlier ones finished
    assert any(c["t_admit"] >= first_done for c in done)
    # and joined while others were still iterating (their work overlapped)
    assert any(a["t_start"] < b["t_start"] < a["t_done"] for a in done for b in done if a is not b)


def test_server_result_same_alone_and_in_mix():
    probs = workload.batch64(8)
    srv = hb.hubbard_server_create(1 << 30, 8)
    ids = [_submit(srv, p) for p in probs]
    mix = _collect(srv, len(ids))
    hb.hubbard_server_destroy(srv)
    for k in (0, 5):
        srv1 = hb.hubbard_server_create(1 << 30, 1)
        rid = _submit(srv1, probs[k])
        alone = _collect(srv1, 1)[rid]
        hb.hubbard_server_destroy(srv1)
        assert alone["E0"] == mix[ids[k]]["E0"] and alone["n_iter"] == mix[ids[k]]["n_iter"]


def test_server_large_sector_on_second_stream():
    """Sectors whose rows exceed the batched kernels' 64 KB run on the solo
    executor's stream beside small batched ones: a 17-site ring with 1 up and
    8 down electrons (rows of 24,310 FP32 values, 95 KB: the two-pass H.v) and
    an 18-site ring with 1 up and 9 down (rows of 48,620 values, wider than the
    LDS: the one-pass H.v).  Every result, the solo ones included, is checked
    against the oracle's E0 from the same seed."""
    solo = [workload.problem("ring17_1u8d", 17, workload.ring(17), 1, 8, 1.0, 5.0),
            workload.problem("ring18_1u9d", 18, workload.ring(18), 1, 9, 1.0, 4.0, seed=11)]
    small = workload.batch64(4)
    srv = hb.hubbard_server_create(4 << 30, 8)
    solo_ids = {_submit(srv, p): p for p in solo}
    ids = {_submit(srv, p): p for p in small}
    res = _collect(srv, len(solo_ids) + len(ids))
    st = hb.hubbard_server_stats(srv)
    hb.hubbard_server_destroy(srv)
    assert st["solo_runs"] == len(solo)
    for rid, p in list(solo_ids.items()) + list(ids.items()):
        assert res[rid]["status"] == hb.HUBBARD_OK, p.name
        assert res[rid]["E0"] == pytest.approx(_oracle_e0(p), rel=1e-6), p.name


def test_server_rejects_malformed_requests():
    srv = hb.hubbard_server_create(1 << 20, 2)
    with pytest.raises(hb.HubbardError):
        hb.hubbard_server_submit(srv, 0, [], 0, 0)
    with pytest.raises(hb.HubbardError):
        hb.hubbard_server_submit(srv, 4, workload.ring(4), 2, 2, max_iter=0)
    hb.hubbard_server_destroy(srv)
