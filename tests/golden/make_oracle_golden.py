"""Write the oracle's Lanczos results for the large sectors to JSON fixtures.

Calls only the oracle (``oracle/``) on the seeded workloads of ``workload``.
Run from the repository root:  python tests/golden/make_oracle_golden.py [ring14|square4x4]
The 4x4 sector takes about an hour on one core (15 s per H.v).
"""
import json
import os
import platform
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
import workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(p, tol, max_iter, want_psi):
    t0 = time.time()
    m = oracle.Model(p.sites, p.edges, p.n_up, p.n_dn, p.t, p.U)
    f1 = oracle.start_vector(p.seed, m.dim)
    r = m.lanczos(f1, tol=tol, max_iter=max_iter, want_psi=want_psi)
    out = {
        "problem": {"name": p.name, "sites": p.sites, "edges": [list(e) for e in p.edges], "n_up": p.n_up,
                    "n_dn": p.n_dn, "t": p.t, "U": p.U, "seed": p.seed, "dim": m.dim},
        "start_vector": "SplitMix64 counter J+1 from the seed, 2u-1, normalised in FP64",
        "tol": tol, "max_iter": max_iter, "n_iter": r["n_iter"], "converged": r["converged"],
        "E0": r["E0"], "a": list(r["a"]), "b": list(r["b"]), "e_hist": list(r["e_hist"]),
        "seconds": time.time() - t0, "host": platform.processor() or platform.machine(),
    }
    if want_psi:
        out.update(residual=r["residual"], rayleigh=r["rayleigh"])
    return out


def main(which):
    if which == "ring14":
        res = run(workload.ring14(), 1e-12, 400, True)
    elif which == "square4x4":
        res = run(workload.square4x4(), -1.0, 200, False)
    else:
        raise SystemExit("unknown workload " + which)
    path = os.path.join(HERE, "oracle_%s.json" % which)
    with open(path, "w") as fh:
        json.dump(res, fh, indent=1)
    print(path, res["n_iter"], res["E0"], "%.1fs" % res["seconds"])


if __name__ == "__main__":
    main(sys.argv[1])
