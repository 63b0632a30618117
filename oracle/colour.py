"""Exact colour matrices for g g -> t tbar + n g -- oracle side (test infrastructure).

The colour basis of an amplitude with one quark line and gluons 1..m is the
set of m! products (T^{a_s1} ... T^{a_sm})_{i j}, one per ordering s
(lexicographic order of the permutations of 0..m-1).  The colour matrix is

    CF[s][r] = sum over all colours of (T^s)_{ij} conj((T^r)_{ij})
             = Tr(T^{s1} ... T^{sm} T^{rm} ... T^{r1}),

evaluated exactly with the SU(N) Fierz identities (T^a = lambda^a / 2):

    Tr(T^a X T^a Y)      = 1/2 [Tr(X) Tr(Y) - Tr(X Y) / N]
    Tr(T^a X) Tr(T^a Y)  = 1/2 [Tr(X Y)     - Tr(X) Tr(Y) / N]
    Tr(1)                = N = 3.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import permutations

NC = 3


def _rotate(tr, k):
    return tr[k:] + tr[:k]


@lru_cache(maxsize=None)
def trace_value(traces):
    """Sum over repeated adjoint labels of a product of traces.

    `traces` is a tuple of tuples of labels; every label occurs exactly twice in
    the whole product."""
    traces = tuple(traces)
    # find a label
    for ti, tr in enumerate(traces):
        if tr:
            a = tr[0]
            break
    else:
        return Fraction(NC) ** len(traces)
    pos = [(ti, k) for ti, tr in enumerate(traces) for k, x in enumerate(tr) if x == a]
    assert len(pos) == 2, "each label must occur twice"
    (t1, k1), (t2, k2) = pos
    rest = [tr for i, tr in enumerate(traces) if i not in (t1, t2)]
    half = Fraction(1, 2)
    if t1 == t2:
        tr = _rotate(traces[t1], k1)          # T^a X T^a Y
        j = tr.index(a, 1)
        X, Y = tr[1:j], tr[j + 1:]
        return half * (trace_value(tuple(rest + [X, Y]))
                       - Fraction(1, NC) * trace_value(tuple(rest + [X + Y])))
    X = _rotate(traces[t1], k1)[1:]           # Tr(T^a X)
    Y = _rotate(traces[t2], k2)[1:]           # Tr(T^a Y)
    return half * (trace_value(tuple(rest + [X + Y]))
                   - Fraction(1, NC) * trace_value(tuple(rest + [X, Y])))


def orderings(m):
    return list(permutations(range(m)))


def colour_matrix(m):
    """Exact colour matrix (list of lists of Fractions) for m gluons."""
    words = orderings(m)
    cf = []
    for s in words:
        row = []
        for r in words:
            row.append(trace_value((tuple(s) + tuple(reversed(r)),)))
        cf.append(row)
    return cf


def colour_matrix_float(m):
    import numpy as np
    return np.array([[float(x) for x in row] for row in colour_matrix(m)], dtype=np.float64)
