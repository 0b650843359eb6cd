"""Independent references the oracle is pinned to (no GPU, no oracle code).

Each helper here derives shortest-path facts by a route other than the
Floyd-Warshall triple loop: brute-force path enumeration, the Bellman
optimality condition, closed forms, a library routine.  The pin tests and
the mutation test both use them.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

INF = 1 << 30


def brute_force(W, inf=INF):
    """Shortest simple-path lengths by enumerating every simple path (tiny n).
    Returns (dist, unique) where unique[i][j] marks a single optimal path, and
    first[i][j] its first hop (or -1)."""
    n = len(W)
    absent = (lambda w: w >= inf) if isinstance(inf, int) else (lambda w: math.isinf(w))
    best = [[None] * n for _ in range(n)]
    count = [[0] * n for _ in range(n)]
    first = [[-1] * n for _ in range(n)]
    for i in range(n):
        best[i][i] = 0
        count[i][i] = 1
        first[i][i] = i
        stack = [(i, 0, (i,))]
        while stack:
            u, d, path = stack.pop()
            for v in range(n):
                if v in path or absent(W[u][v]):
                    continue
                nd = d + W[u][v]
                if best[i][v] is None or nd < best[i][v]:
                    best[i][v] = nd
                    count[i][v] = 1
                    first[i][v] = path[1] if len(path) > 1 else v
                elif nd == best[i][v]:
                    count[i][v] += 1
                stack.append((v, nd, path + (v,)))
    dist = [[(inf if best[i][j] is None else best[i][j]) for j in range(n)] for i in range(n)]
    unique = [[count[i][j] == 1 for j in range(n)] for i in range(n)]
    return dist, unique, first


def bellman_first_hop(W, D):
    """For graphs with unique shortest paths: the successor of i towards j is
    the h minimising W[i][h] + D[h][j] over edges i -> h (float64)."""
    n = D.shape[0]
    Wf = W.astype(np.float64).copy()
    np.fill_diagonal(Wf, np.inf)
    Df = D.astype(np.float64)
    nx = np.full((n, n), -1, np.int64)
    for i in range(n):
        cand = Wf[i][:, None] + Df          # cand[h, j] = W[i][h] + D[h][j]
        nx[i] = np.argmin(cand, axis=0)
        nx[i, i] = i
    nx[~np.isfinite(Df)] = -1
    return nx


def reachability(W, absent_mask):
    """Transitive closure of the edge relation by repeated boolean squaring."""
    n = W.shape[0]
    R = (~absent_mask) | np.eye(n, dtype=bool)
    while True:
        R2 = R | ((R.astype(np.int64) @ R.astype(np.int64)) > 0)
        if (R2 == R).all():
            return R
        R = R2


def scipy_dist(W, absent_mask):
    """Library routine: scipy's Dijkstra on a sparse graph (zero weights kept)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    n = W.shape[0]
    ii, jj = np.nonzero(~absent_mask & ~np.eye(n, dtype=bool))
    vals = W[ii, jj].astype(np.float64)
    assert (vals > 0).all(), "scipy pin is used with positive weights only"
    g = csr_matrix((vals, (ii, jj)), shape=(n, n))
    return shortest_path(g, method="D", directed=True)


def chain(n, w):
    """Path 0 -> 1 -> ... -> n-1 with weights w[t] on edge t -> t+1."""
    W = np.full((n, n), INF, np.int64)
    np.fill_diagonal(W, 0)
    for t in range(n - 1):
        W[t, t + 1] = w[t]
    D = np.full((n, n), INF, np.int64)
    NX = np.full((n, n), -1, np.int64)
    pre = np.concatenate([[0], np.cumsum(w)])
    for i in range(n):
        for j in range(i, n):
            D[i, j] = pre[j] - pre[i]
            NX[i, j] = i if i == j else i + 1
    return W, D, NX


def cycle(n, w):
    """Directed cycle t -> t+1 (mod n), weights w[t]."""
    W = np.full((n, n), INF, np.int64)
    np.fill_diagonal(W, 0)
    for t in range(n):
        W[t, (t + 1) % n] = w[t]
    D = np.zeros((n, n), np.int64)
    NX = np.zeros((n, n), np.int64)
    for i in range(n):
        s = 0
        for step in range(n):
            j = (i + step) % n
            D[i, j] = s
            NX[i, j] = i if step == 0 else (i + 1) % n
            s += w[j]
    return W, D, NX


def load_golden(path):
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    n = int(lines[0].split()[1])
    idx = lines.index("edges")
    idist = lines.index("dist")
    inext = lines.index("next")
    W = np.full((n, n), INF, np.int64)
    np.fill_diagonal(W, 0)
    for ln in lines[idx + 1:idist]:
        u, v, w = map(int, ln.split())
        W[u, v] = w
    D = np.array([list(map(int, ln.split())) for ln in lines[idist + 1:inext]], np.int64)
    NX = np.array([list(map(int, ln.split())) for ln in lines[inext + 1:inext + 1 + n]], np.int64)
    D[D < 0] = INF
    return W, D, NX


def exhaustive_n3():
    """All 3^6 directed graphs on 3 vertices with weights in {1, 2, absent}."""
    vals = [1, 2, INF]
    off = [(i, j) for i in range(3) for j in range(3) if i != j]
    for combo in itertools.product(vals, repeat=len(off)):
        W = np.zeros((3, 3), np.int64)
        for (i, j), w in zip(off, combo):
            W[i, j] = w
        yield W
