"""Pins of the reference gradient (oracle/grad.c).

The gradient of L = sum(G * D) with respect to the edge weights is pinned by
things other than its own definition:
  - central finite differences of L through the float64 forward oracle (itself
    pinned by test_oracle.py) on graphs whose shortest paths are unique, where
    D is locally linear in W;
  - closed forms on a chain and a directed cycle;
  - absent edges, the diagonal and unreachable pairs get exactly zero;
  - planted mistakes in grad.c (a dropped hop, a transposed edge or upstream
    index, a truncated walk) each fail one of the above.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth


def fd_grad(W, G, edges, eps):
    """Central differences of sum(G * D(W)) for the listed edges, float64."""
    W = np.asarray(W, np.float64)
    fin = None
    out = []
    for (u, v) in edges:
        Lp = Lm = 0.0
        for sgn in (1.0, -1.0):
            Wp = W.copy()
            Wp[u, v] += sgn * eps
            D, _ = oracle.fw_f64(Wp, next_hop=False)
            if fin is None:
                fin = np.isfinite(D)
            assert np.array_equal(np.isfinite(D), fin)
            L = float(np.sum(np.where(fin, G.astype(np.float64) * np.where(fin, D, 0.0), 0.0)))
            if sgn > 0:
                Lp = L
            else:
                Lm = L
        out.append((Lp - Lm) / (2.0 * eps))
    return np.array(out)


def check_against_fd(W, G, lib=None, eps=1e-6, tol=2e-6):
    D, NX = oracle.fw_f64(W)
    ref = oracle.grad_ref(G, NX, lib=lib)
    n = W.shape[0]
    present = [(u, v) for u in range(n) for v in range(n) if u != v and np.isfinite(W[u, v])]
    fd = fd_grad(W, G, present, eps)
    fd2 = fd_grad(W, G, present, eps * 10)     # a crossed tie would show as a disagreement
    np.testing.assert_allclose(fd, fd2, atol=tol)
    got = np.array([ref[u, v] for (u, v) in present])
    bad = np.abs(got - fd) > tol
    # absent edges and the diagonal carry nothing
    absent = ~np.isfinite(np.asarray(W, np.float64))
    np.fill_diagonal(absent, True)
    return int(np.count_nonzero(bad)) + int(np.count_nonzero(ref[absent]))


def fd_graphs():
    # complete graph, weights U[0.5, 1.5): paths of one or two hops
    yield synth.graph_f32(12, 51, 1.0, 0.5, 1.5), synth.normal_f32(12, 12, 52)
    # sparse graph, longer paths and unreachable pairs
    yield synth.graph_f32(16, 53, 0.2, 0.1, 10.0), synth.normal_f32(16, 16, 54)
    # medium density
    yield synth.graph_f32(20, 55, 0.35, 0.1, 10.0), synth.normal_f32(20, 20, 56)
    yield synth.graph_f32(2, 57, 1.0, 0.1, 1.0), synth.normal_f32(2, 2, 58)


@pytest.mark.parametrize("case", range(4))
def test_grad_matches_finite_differences(case):
    W, G = list(fd_graphs())[case]
    assert check_against_fd(W, G) == 0


def test_grad_closed_form_chain_and_cycle():
    n = 9
    # chain 0 -> 1 -> ... -> n-1: edge (k, k+1) lies on the paths i -> j with
    # i <= k < j, i.e. (k + 1) * (n - 1 - k) pairs
    W = np.full((n, n), np.inf, np.float32)
    np.fill_diagonal(W, 0)
    for k in range(n - 1):
        W[k, k + 1] = 1.0 + k
    _, NX = oracle.fw_f64(W)
    g = oracle.grad_ref(np.ones((n, n), np.float32), NX)
    for k in range(n - 1):
        assert g[k, k + 1] == (k + 1) * (n - 1 - k)
    assert np.count_nonzero(g) == n - 1
    # directed cycle: every edge lies on exactly n(n-1)/2 of the n(n-1) paths
    # (path i -> j uses edge (k, k+1 mod n) iff k is among the j - i mod n
    # vertices from i on; summed over pairs that is n (n-1) / 2 per edge)
    W = np.full((n, n), np.inf, np.float32)
    np.fill_diagonal(W, 0)
    for k in range(n):
        W[k, (k + 1) % n] = 2.0
    _, NX = oracle.fw_f64(W)
    g = oracle.grad_ref(np.ones((n, n), np.float32), NX)
    for k in range(n):
        assert g[k, (k + 1) % n] == n * (n - 1) // 2
    # a weighted upstream on the chain: edge (k, k+1) sums G[i][j] over i <= k < j
    W = np.full((n, n), np.inf, np.float32)
    np.fill_diagonal(W, 0)
    for k in range(n - 1):
        W[k, k + 1] = 1.0
    _, NX = oracle.fw_f64(W)
    G = synth.normal_f32(n, n, 60)
    g = oracle.grad_ref(G, NX)
    for k in range(n - 1):
        want = sum(float(G[i, j]) for i in range(k + 1) for j in range(k + 1, n))
        assert abs(g[k, k + 1] - want) < 1e-9


def test_grad_empty_graph_and_broken_walk():
    n = 5
    W = np.full((n, n), np.inf, np.float32)
    np.fill_diagonal(W, 0)
    _, NX = oracle.fw_f64(W)
    assert not oracle.grad_ref(np.ones((n, n), np.float32), NX).any()
    NX = np.array([[0, 1], [0, 1]], np.int32)
    NX[0, 1] = 0                                   # a walk that never reaches 1
    with pytest.raises(ValueError):
        oracle.grad_ref(np.ones((2, 2), np.float32), NX)


GRAD_SRC = os.path.join(os.path.dirname(oracle.__file__), "grad.c")
FW_SRC = os.path.join(os.path.dirname(oracle.__file__), "fw_oracle.c")
VAL_SRC = os.path.join(os.path.dirname(oracle.__file__), "validate.c")

GRAD_MUTANTS = {
    "last hop dropped": ("while (u != j) {", "while (NX[u * ld + j] != j) {"),
    "edge transposed": ("out[u * ldo + h] += g;", "out[h * ldo + u] += g;"),
    "upstream transposed": ("(double)G[i * ldg + j];", "(double)G[j * ldg + i];"),
    "first hop only": ("        u = h;\n                ++hops;", "        u = j;\n                ++hops;"),
    "walk toward the source": ("const int64_t h = NX[u * ld + j];", "const int64_t h = NX[u * ld + i];"),
}


@pytest.mark.parametrize("name", sorted(GRAD_MUTANTS))
def test_grad_mutant_is_caught(name, tmp_path):
    old, new = GRAD_MUTANTS[name]
    src = open(GRAD_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not found"
    cfile = tmp_path / "grad_mut.c"
    cfile.write_text(src.replace(old, new))
    so = tmp_path / "libgradmut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           FW_SRC, VAL_SRC, str(cfile), "-o", str(so), "-lm"])
    lib = oracle.load_library(str(so))
    caught = 0
    for W, G in fd_graphs():
        try:
            caught += check_against_fd(W, G, lib=lib)
        except ValueError:
            caught += 1
    assert caught, f"planted mistake {name!r} passed every gradient pin"
