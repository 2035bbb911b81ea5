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
    """A sector above the batched size runs on the two-pass path beside small
    ones; its mixed-precision E0 agrees with the FP64 single-instance path."""
    big = workload.problem("sq4x4_5u5d", 16, workload.torus(4, 4), 5, 5, 1.0, 6.0)
    small = workload.batch64(4)
    srv = hb.hubbard_server_create(4 << 30, 8)
    big_id = _submit(srv, big)
    ids = {_submit(srv, p): p for p in small}
    res = _collect(srv, 1 + len(ids))
    hb.hubbard_server_destroy(srv)
    h = hb.hubbard_build(big.sites, big.edges, big.n_up, big.n_dn, big.t, big.U)
    ref = hb.hubbard_lanczos_ex(h, tol=1e-12, max_iter=300, precision=hb.HUBBARD_FP64, seed=big.seed)
    assert res[big_id]["status"] == hb.HUBBARD_OK
    assert res[big_id]["E0"] == pytest.approx(ref["E0"], rel=1e-6)
    for rid, p in ids.items():
        assert res[rid]["E0"] == pytest.approx(_oracle_e0(p), rel=1e-6)


def test_server_rejects_malformed_requests():
    srv = hb.hubbard_server_create(1 << 20, 2)
    with pytest.raises(hb.HubbardError):
        hb.hubbard_server_submit(srv, 0, [], 0, 0)
    with pytest.raises(hb.HubbardError):
        hb.hubbard_server_submit(srv, 4, workload.ring(4), 2, 2, max_iter=0)
    hb.hubbard_server_destroy(srv)
