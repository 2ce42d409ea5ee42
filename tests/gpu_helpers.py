"""Shared helpers of the GPU parity tests (comparisons against the CPU oracle)."""
import sys

import numpy as np

import oracle
import paper_2606_26760_amd as hq


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solver_for(ints, alpha, beta, na, nb):
    s = hq.Hinqs()
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(alpha, beta, na, nb)
    return s


def oracle_for(ints, alpha, beta, na, nb):
    return oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)


def gpu_rows_as_tuples(solver, rows):
    """Per requested caller row: sorted list of (j, type, h1, h2, p1, p2, neg)."""
    rowptr, col, desc = solver.connectivity()
    rowptr = rowptr.cpu().numpy()
    col = col.cpu().numpy()
    desc = desc.cpu().numpy().view(np.uint32)
    t, neg, h1, h2, p1, p2 = hq.decode_descriptor(desc)
    out = {}
    for i in rows:
        a, b = rowptr[i], rowptr[i + 1]
        items = []
        for e in range(a, b):
            typ = int(t[e])
            if typ in (hq.EXC_1A, hq.EXC_1B):
                items.append((int(col[e]), typ, int(h1[e]), -1, int(p1[e]), -1, int(neg[e])))
            else:
                items.append((int(col[e]), typ, int(h1[e]), int(h2[e]), int(p1[e]), int(p2[e]),
                              int(neg[e])))
        out[int(i)] = sorted(items)
    return out


def oracle_rows_as_tuples(orc, rows):
    r = orc.rows(rows)
    out = {}
    for t, i in enumerate(r["rows"]):
        items = []
        for e in range(r["rowptr"][t] + 1, r["rowptr"][t + 1]):
            o = [int(v) for v in r["orb"][e]]
            items.append((int(r["col"][e]), int(r["etype"][e]), o[0], o[1], o[2], o[3],
                          1 if r["sign"][e] < 0 else 0))
        out[int(i)] = sorted(items)
    return out, r


def row_bound(r, X, k):
    """Per sampled row: sum_j |H_ij| |X_j| (cancellation-safe scale of the row sum)."""
    nr = len(r["rows"])
    b = np.zeros((nr, k))
    for t in range(nr):
        a, e = r["rowptr"][t], r["rowptr"][t + 1]
        b[t] = (np.abs(r["val"][a:e])[:, None] * np.abs(X[r["col"][a:e]])).sum(axis=0)
    return b
