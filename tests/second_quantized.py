"""Independent brute-force Hubbard Hamiltonian for tiny lattices (tests only).

Built directly from the operator algebra of Sec. 1-2.1 of Siro & Harju: a
basis state is the ordered string of creation operators acting on the vacuum
(all up operators left of all down operators, sites ascending, eq. basisstate).
A hop c^dag_{a s} c_{b s} is applied by literally anticommuting the
annihilator to its partner and the new creator to its canonical place,
counting one -1 per operator passed.  No bit tricks and no per-spin
factorisation are used, so it checks the oracle's sign rule and its J order
independently.  The states are labelled by J = i_up * dim_dn + i_dn with
i_sigma the position of the configuration in ascending integer order
(eq. J-formula), computed here from Python's sorted() over combinations.
"""
import itertools

import numpy as np


def _configs(ns, n):
    words = sorted(sum(1 << s for s in c) for c in itertools.combinations(range(ns), n))
    return words


def _ops(up_word, dn_word, ns):
    """Canonical operator string: list of (spin, site), spin 0 = up first."""
    return [(0, s) for s in range(ns) if (up_word >> s) & 1] + [(1, s) for s in range(ns) if (dn_word >> s) & 1]


def _canonical_key(op):
    return (op[0], op[1])


def _hop(ops, spin, a, b):
    """c^dag_{a,spin} c_{b,spin} |ops>  ->  (sign, new_ops) or None."""
    if (spin, b) not in ops:
        return None
    p = ops.index((spin, b))
    sign = (-1) ** p  # move the annihilator past p creators, then {c_b, c^dag_b} = 1
    rest = ops[:p] + ops[p + 1:]
    if (spin, a) in rest:
        return None  # (c^dag)^2 = 0
    # place c^dag_a at the front, then anticommute it to its canonical place
    q = sum(1 for op in rest if _canonical_key(op) < (spin, a))
    sign *= (-1) ** q
    new = rest[:q] + [(spin, a)] + rest[q:]
    return sign, new


def dense_hamiltonian(ns, edges, n_up, n_dn, t, U):
    """t: one amplitude for all bonds, or one per bond (in the order of edges)."""
    amps = [t] * len(edges) if np.ndim(t) == 0 else list(t)
    ups, dns = _configs(ns, n_up), _configs(ns, n_dn)
    iu = {w: k for k, w in enumerate(ups)}
    idn = {w: k for k, w in enumerate(dns)}
    dim = len(ups) * len(dns)
    H = np.zeros((dim, dim))
    for wu in ups:
        for wd in dns:
            J = iu[wu] * len(dns) + idn[wd]
            ops = _ops(wu, wd, ns)
            # interaction: U n_{i up} n_{i dn}
            H[J, J] += U * sum(1 for s in range(ns) if (0, s) in ops and (1, s) in ops)
            # hopping: -t sum_<ij> sum_s (c^dag_i c_j + c^dag_j c_i)
            for (i, j), tb in zip(edges, amps):
                for spin in (0, 1):
                    for (a, b) in ((i, j), (j, i)):
                        r = _hop(ops, spin, a, b)
                        if r is None:
                            continue
                        sign, new = r
                        nu = sum(1 << s for (sp, s) in new if sp == 0)
                        nd = sum(1 << s for (sp, s) in new if sp == 1)
                        J2 = iu[nu] * len(dns) + idn[nd]
                        H[J2, J] += -tb * sign
    return H
