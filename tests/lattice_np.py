"""Test-side lattice helpers, independent of the oracle's C code: shells of Z^5 by
direct enumeration, coordinates (x0 fastest), and cluster labels of an occupied
set by scipy's connected_components (a library graph routine)."""
import itertools

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def shell_offsets(mask):
    out = []
    for d in itertools.product(range(-2, 3), repeat=5):
        r2 = sum(x * x for x in d)
        if 1 <= r2 <= 7 and mask & (1 << (r2 - 1)):
            out.append(d)
    return np.array(out, dtype=np.int64).reshape(-1, 5)


def coords(L, sites):
    sites = np.asarray(sites, dtype=np.int64)
    return np.stack([(sites // L**j) % L for j in range(5)], axis=-1)


def components(L, mask, occupied_sites, periodic=False):
    """Labels (smallest member index; -1 for empty) of the clusters formed by the
    occupied sites under the zone-mask neighbourhood with free (or periodic:
    coordinates mod L) boundaries."""
    N = L**5
    occ = np.zeros(N, dtype=bool)
    occ[np.asarray(occupied_sites, dtype=np.int64)] = True
    idx = np.nonzero(occ)[0]
    x = coords(L, idx)
    rows, cols = [], []
    for d in shell_offsets(mask):
        y = x + d
        if periodic:
            y = np.mod(y, L)
        inb = ((y >= 0) & (y < L)).all(axis=1)
        t = (y[inb] * (L ** np.arange(5))).sum(axis=1)
        ok = occ[t]
        rows.append(idx[inb][ok])
        cols.append(t[ok])
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    _, lab = connected_components(g, directed=False)
    out = np.full(N, -1, dtype=np.int64)
    # canonical label: smallest site index in the component
    comp_min = {}
    for i in idx:
        c = lab[i]
        if c not in comp_min:
            comp_min[c] = i
    for i in idx:
        out[i] = comp_min[lab[i]]
    return out


def spans(L, labels):
    """True if some cluster has members at x0 = 0 and at x0 = L-1."""
    occ = np.nonzero(labels >= 0)[0]
    if len(occ) == 0:
        return False
    x0 = occ % L
    lo = set(labels[occ[x0 == 0]].tolist())
    hi = set(labels[occ[x0 == L - 1]].tolist())
    return bool(lo & hi)


def wrapping_roots(L, mask, occupied_sites):
    """Labels (as in components) of the clusters that wrap around axis 0 on the
    periodic lattice (L >= 5), and the cluster sizes, by breadth-first search:
    each cluster gets unwrapped x0 coordinates along a BFS tree, and it wraps iff
    some edge t = s + d of it has u(t) != u(s) + d0 (the loop that edge closes
    winds around axis 0).  Independent of any union-find."""
    from collections import deque

    assert L >= 5
    N = L**5
    occ = np.zeros(N, dtype=bool)
    occ[np.asarray(occupied_sites, dtype=np.int64)] = True
    offs = shell_offsets(mask)
    strides = L ** np.arange(5)

    def nbrs(s):
        y = np.mod(coords(L, [s])[0] + offs, L)
        t = (y * strides).sum(axis=1)
        keep = occ[t]
        return t[keep], offs[keep, 0]

    u = {}
    size = {}
    wraps = set()
    for start in np.nonzero(occ)[0]:
        start = int(start)
        if start in u:
            continue
        u[start] = 0
        q = deque([start])
        members = 0
        bad = False
        while q:
            s = q.popleft()
            members += 1
            ts, d0s = nbrs(s)
            for t, d0 in zip(ts.tolist(), d0s.tolist()):
                if t not in u:
                    u[t] = u[s] + d0
                    q.append(t)
                elif u[t] != u[s] + d0:
                    bad = True
        size[start] = members
        if bad:
            wraps.add(start)
    return wraps, size


def first_wrap(L, mask, order):
    """(n*, mass) of the first cluster wrapping around axis 0 along the order
    (0, 0 if none within it), by bisection on n (wrapping is monotone: a
    cluster only grows and a loop once formed stays)."""
    order = np.asarray(order)

    def wrapped(n):
        w, _ = wrapping_roots(L, mask, order[:n])
        return bool(w)

    if len(order) == 0 or not wrapped(len(order)):
        return 0, 0
    lo, hi = 0, len(order)      # wrapped(lo) false, wrapped(hi) true
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if wrapped(mid):
            hi = mid
        else:
            lo = mid
    w, size = wrapping_roots(L, mask, order[:hi])
    assert len(w) == 1
    return hi, size[next(iter(w))]
