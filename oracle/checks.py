"""Brute-force checkers that pin the oracle (test infrastructure only).

These are written independently of ``oracle.c`` and of the GPU path, in
NumPy, for small inputs:

* ``kruskal_full``: Kruskal over the full key matrix (every unordered pair,
  sorted by (s, i, j)).  The key-ordered minimum spanning tree is unique, so
  Prim in the oracle must return the same edge set, bit for bit.
* ``path_max_matrix`` / ``cycle_property_violations``: for a spanning tree,
  the largest key on the tree path between every pair; a tree is the minimum
  spanning tree iff every non-tree pair has a larger key than that.
* ``eps_components``: connected components of the graph that joins every
  pair with sqrt(s) <= dmax (the distance-threshold cut with nothing else on).
* ``agglo_allpairs``: the paper's own process over all pairs of points: at
  every step take, among admissible cluster pairs, the smallest (class,
  single-link key) and unite, until KL1 is reached or nothing is admissible.
* ``canonical``: relabel in order of first appearance.
"""
from __future__ import annotations

import numpy as np


def key_matrix(X):
    """FP64 squared distances, each feature widened exactly from FP32,
    differences and squares rounded once, added in feature order."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    n, d = X.shape
    s = None
    for f in range(d):
        diff = X[:, f][:, None] - X[:, f][None, :]
        sq = diff * diff
        s = sq if s is None else s + sq
    return s


def _find(par, x):
    while par[x] != x:
        par[x] = par[par[x]]
        x = par[x]
    return x


def kruskal_full(X):
    """Edges (u, v, s) of the key-ordered MST, sorted by key."""
    S = key_matrix(X)
    n = S.shape[0]
    iu, ju = np.triu_indices(n, 1)
    sv = S[iu, ju]
    order = np.lexsort((ju, iu, sv))
    par = list(range(n))
    out = []
    for e in order:
        a, b = int(iu[e]), int(ju[e])
        ra, rb = _find(par, a), _find(par, b)
        if ra != rb:
            par[ra] = rb
            out.append((a, b, float(sv[e])))
            if len(out) == n - 1:
                break
    u = np.array([e[0] for e in out], np.int32)
    v = np.array([e[1] for e in out], np.int32)
    s = np.array([e[2] for e in out], np.float64)
    return u, v, s


def key_less(a, b):
    """Lexicographic (s, lo, hi) compare of two key tuples."""
    return tuple(a) < tuple(b)


def path_max_matrix(n, u, v):
    """M[i, j] = index (in the given key order) of the largest tree edge on
    the path from i to j; -1 on the diagonal.  Edges must be key-sorted."""
    M = np.full((n, n), -1, dtype=np.int64)
    members = {i: [i] for i in range(n)}
    root = list(range(n))
    for e in range(len(u)):
        ra, rb = root[int(u[e])], root[int(v[e])]
        A, B = members[ra], members[rb]
        ia = np.array(A)
        ib = np.array(B)
        M[np.ix_(ia, ib)] = e
        M[np.ix_(ib, ia)] = e
        if len(A) < len(B):
            ra, rb, A, B = rb, ra, B, A
        A.extend(B)
        for x in B:
            root[x] = ra
        del members[rb]
    return M


def cycle_property_violations(X, u, v, s):
    """Number of non-tree pairs whose key is not larger than the largest
    key on their tree path (0 iff the tree is the key-ordered MST)."""
    S = key_matrix(X)
    n = S.shape[0]
    M = path_max_matrix(n, u, v)
    iu, ju = np.triu_indices(n, 1)
    e = M[iu, ju]
    es, eu, ev = s[e], u[e], v[e]
    ps = S[iu, ju]
    tree = (iu == eu) & (ju == ev)
    larger = (ps > es) | ((ps == es) & ((iu > eu) | ((iu == eu) & (ju > ev))))
    return int(np.count_nonzero(~tree & ~larger))


def canonical(labels):
    labels = np.asarray(labels)
    out = np.empty(labels.shape[0], np.int32)
    seen = {}
    for i, l in enumerate(labels.tolist()):
        if l not in seen:
            seen[l] = len(seen)
        out[i] = seen[l]
    return out


def eps_components(X, dmax):
    S = key_matrix(X)
    A = np.sqrt(S) <= dmax
    n = A.shape[0]
    lab = np.full(n, -1, np.int64)
    c = 0
    for i in range(n):
        if lab[i] >= 0:
            continue
        stack = [i]
        lab[i] = c
        while stack:
            x = stack.pop()
            for y in np.nonzero(A[x] & (lab < 0))[0].tolist():
                lab[y] = c
                stack.append(y)
        c += 1
    return canonical(lab), c


def drop_heaviest(n, u, v, k):
    """Components left after removing the k-1 largest-key tree edges."""
    par = list(range(n))
    keep = len(u) - (k - 1) if k >= 1 else len(u)
    for e in range(max(keep, 0)):
        ra, rb = _find(par, int(u[e])), _find(par, int(v[e]))
        if ra != rb:
            par[ra] = rb
    return canonical([_find(par, i) for i in range(n)])


def agglo_allpairs(X, kl1=0, kl2=-1, kl3=-1, kl4=0, dmax=float("inf")):
    """The paper's process over all pairs of points (slow; small n only)."""
    S = key_matrix(X)
    n = S.shape[0]
    W = np.sqrt(S)
    lab = np.arange(n)
    while True:
        ids = np.unique(lab)
        if kl1 > 0 and len(ids) <= kl1:
            break
        size = {c: int(np.count_nonzero(lab == c)) for c in ids.tolist()}
        best = None
        for a_i, a in enumerate(ids.tolist()):
            ia = np.nonzero(lab == a)[0]
            for b in ids.tolist()[a_i + 1:]:
                ib = np.nonzero(lab == b)[0]
                sub = S[np.ix_(ia, ib)]
                # single-link key between the two clusters
                flat = []
                for x_k, x in enumerate(ia.tolist()):
                    for y_k, y in enumerate(ib.tolist()):
                        flat.append((sub[x_k, y_k], min(x, y), max(x, y)))
                key = min(flat)
                w = float(np.sqrt(key[0]))
                sa, sb = size[a], size[b]
                if w > dmax:
                    continue
                if kl2 >= 0 and max(sa, sb) > kl2:
                    continue
                if kl3 >= 0 and sa + sb > kl3:
                    continue
                cls = 0 if (kl4 > 1 and min(sa, sb) < kl4) else 1
                cand = (cls, key, a, b)
                if best is None or cand[:2] < best[:2]:
                    best = cand
        if best is None:
            break
        _, _, a, b = best
        lab[lab == b] = a
    del W
    return canonical(lab), len(np.unique(lab))
