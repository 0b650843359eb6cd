"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

The oracle is the plain Floyd-Warshall loop (Section 2.3, Fig. 1).  Nothing
here re-types its loop: every expected value comes from brute-force path
enumeration, Dijkstra, scipy, the Bellman optimality condition, closed
forms, a hand-worked fixture or an invariant.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pins as P

INF = P.INF
HERE = os.path.dirname(os.path.abspath(__file__))


def rand_graph(n, seed, p, lo, hi):
    return synth.graph_i32(n, seed, p, lo, hi)


def check_all_pins_i32(W, lib=None, unique_check=False):
    """Run every pin that applies to an int32 graph; returns a list of failures."""
    fails = []
    n = W.shape[0]
    D, NX = oracle.fw_i32(W, lib=lib)
    Wn = np.where(W >= INF, INF, W).astype(np.int64)
    np.fill_diagonal(Wn, 0)
    absent = Wn >= INF
    # 1. Dijkstra from every source
    Rd = oracle.sssp_i32(W, np.arange(n))
    if not (Rd == D).all():
        fails.append("dijkstra")
    # 2. invariants
    if (np.diag(D) != 0).any():
        fails.append("diag")
    if (D > Wn).any():
        fails.append("D<=W")
    if oracle.triangle_violations(D) != 0:
        fails.append("triangle")
    R = P.reachability(Wn, absent)
    if ((D < INF) != R).any():
        fails.append("reachability")
    bad, first = oracle.validate_walk(W, D, NX)
    if bad:
        fails.append(f"walk {first}")
    return fails, D, NX


def _broken_cases(W, D, NX, inf):
    """Plausible wrong (D, NX) pairs derived from a correct one, each with the
    validator's reason code and the pair it must name first."""
    n = D.shape[0]
    fin = np.isfinite(D) if D.dtype.kind == "f" else (D < inf)
    cases = []
    D1 = D.copy(); D1[0, 0] = 1
    cases.append(("nonzero diagonal", D1, NX, (0, 0, 1)))
    N1 = NX.copy(); N1[1, 1] = 0
    cases.append(("diagonal successor", D, N1, (1, 1, 1)))
    i, j = [int(x) for x in np.argwhere(fin & ~np.eye(n, dtype=bool))[0]]
    N2 = NX.copy(); N2[i, j] = -1
    cases.append(("finite distance without successor", D, N2, (i, j, 2)))
    D2 = D.copy(); D2[i, j] = inf
    cases.append(("infinite distance with a successor", D2, NX, (i, j, 2)))
    if D.dtype.kind == "f":
        D3 = D.copy(); D3[i, j] = -np.inf
        cases.append(("negative infinite distance", D3, NX, (i, j, 2)))
        N3b = NX.copy(); N3b[i, j] = -1
        cases.append(("negative infinite distance without successor", D3, N3b, (i, j, 2)))
    N3 = NX.copy(); N3[i, j] = i
    cases.append(("walk that stays put", D, N3, (i, j, 3)))
    N4 = NX.copy(); N4[i, j] = n
    cases.append(("successor out of range", D, N4, (i, j, 3)))
    # a walk that loops: i -> h -> i -> ... toward j (both hops are edges)
    h = next(v for v in range(n) if v not in (i, j))
    N5 = NX.copy(); N5[i, j] = h; N5[h, j] = i
    cases.append(("walk that loops", D, N5, (min(i, h), j, 3)))
    D6 = D.copy()
    D6[i, j] = D6[i, j] * 1.001 + (1 if D.dtype.kind != "f" else 0)
    cases.append(("sum differs", D6, NX, (i, j, 4)))
    return cases


def check_validator_pins(kind, lib=None):
    """The walk validator must accept correct outputs (closed forms and the
    pinned oracle's) and reject each broken variant with its reason code.
    Returns a list of failures (empty when every pin holds)."""
    fails = []
    n = 12
    rtol = 1e-5
    if kind == "i32":
        W = synth.graph_i32(n, 61, 1.0, 1, 100)
        D, NX = oracle.fw_i32(W)
        inf = INF
        Wc, Dc, NXc = P.chain(n, np.arange(1, n))
        Wc, Dc, NXc = Wc.astype(np.int32), Dc.astype(np.int32), NXc.astype(np.int32)
    else:
        W = synth.graph_f32(n, 61, 1.0, 0.5, 1.5)
        D, NX = oracle.fw_f64(W)
        inf = np.inf
        Wc, Dc, NXc = P.chain(n, np.arange(1, n))
        Wc = np.where(Wc >= INF, np.inf, Wc)
        Dc = np.where(Dc >= INF, np.inf, Dc)
        NXc = NXc.astype(np.int32)
        if kind == "f32":
            W, D, Wc, Dc = W.astype(np.float32), D.astype(np.float32), Wc.astype(np.float32), Dc.astype(np.float32)
        else:
            W, Wc = W.astype(np.float64), Wc.astype(np.float64)
    # acceptance: the oracle's answer, the closed-form chain, and a sum off by
    # less than the tolerance
    if oracle.validate_walk(W, D, NX, rtol=rtol, lib=lib)[0] != 0:
        fails.append("rejects a correct answer")
    if oracle.validate_walk(Wc, Dc, NXc, rtol=rtol, lib=lib)[0] != 0:
        fails.append("rejects the closed-form chain")
    if kind != "i32":
        Dn = D.copy()
        Dn[0, 5] = Dn[0, 5] * (1 + rtol / 4)
        if oracle.validate_walk(W, Dn, NX, rtol=rtol, lib=lib)[0] != 0:
            fails.append("rejects a sum within the tolerance")
    for name, Db, Nb, exp in _broken_cases(W, D, NX, inf):
        bad, first = oracle.validate_walk(W, Db, Nb, rtol=rtol, lib=lib)
        if bad < 1 or first != exp:
            fails.append(f"{name}: got {bad} bad, first {first}, expected {exp}")
    # a hop over an absent edge: on the chain 0 -> 1 -> 2, claim 0 -> 2 directly
    Nb = NXc.copy(); Nb[0, 2] = 2
    bad, first = oracle.validate_walk(Wc, Dc, Nb, rtol=rtol, lib=lib)
    if bad < 1 or first != (0, 2, 3):
        fails.append(f"walk over an absent edge: got {bad}, {first}")
    return fails


@pytest.mark.parametrize("kind", ["i32", "f32", "f64"])
def test_validator_pins(kind):
    """Every reason code of the walk validator, for each element type."""
    fails = check_validator_pins(kind)
    assert not fails, fails


def test_f32_oracle_successor_unique_paths():
    """Float32 oracle on continuous weights (complete graph, U[0.5, 1.5):
    unique shortest paths almost surely).  Distances against float64
    Dijkstra within float32 rounding of a few hops; successors equal the
    Bellman first hop except where the oracle's choice is itself shortest
    within that rounding (a float32 near-tie)."""
    fails = check_f32_oracle_pins()
    assert not fails, fails


def check_f32_oracle_pins(lib=None):
    fails = []
    # integer-valued float weights: every sum is exact
    Wi = synth.graph_i32(90, 62, 0.3, 1, 50)
    Wf = np.where(Wi >= INF, np.inf, Wi).astype(np.float32)
    D32, N32 = oracle.fw_f32(Wf, lib=lib)
    R = oracle.sssp_i32(Wi, np.arange(90))
    if not (D32 == np.where(R >= INF, np.inf, R).astype(np.float32)).all():
        fails.append("integer-valued distances differ from Dijkstra")
    if oracle.validate_walk(Wf, D32, N32, rtol=0.0)[0] != 0:
        fails.append("integer-valued walks")
    # continuous weights
    n = 120
    W = synth.graph_f32(n, 63, 1.0, 0.5, 1.5)
    D32, N32 = oracle.fw_f32(W, lib=lib)
    Dd = oracle.sssp_f64(W, np.arange(n))
    rt = 4 * 2.0 ** -24                      # paths have at most ~3 hops here
    if not (np.abs(D32 - Dd) <= rt * Dd).all():
        fails.append("continuous distances beyond float32 rounding")
    B = P.bellman_first_hop(W, Dd)
    diff = np.argwhere(N32 != B)
    Wd = W.astype(np.float64)
    for i, j in diff:
        h = N32[i, j]
        if h < 0 or i == j or abs(Wd[i, h] + Dd[h, j] - Dd[i, j]) > rt * Dd[i, j]:
            fails.append(f"successor ({i}, {j}) = {h}, Bellman {B[i, j]}")
            break
    if len(diff) > n * n // 1000:
        fails.append(f"{len(diff)} successors differ from the Bellman first hop")
    if oracle.validate_walk(W, D32, N32, rtol=1e-6)[0] != 0:
        fails.append("continuous walks")
    return fails


def test_hand_worked_fixture():
    W, Dg, NXg = P.load_golden(os.path.join(HERE, "golden", "hand_5.txt"))
    D, NX = oracle.fw_i32(W)
    np.testing.assert_array_equal(D, Dg)
    np.testing.assert_array_equal(NX, NXg)
    dist, unique, first = P.brute_force(W.tolist())
    np.testing.assert_array_equal(np.array(dist), Dg)


def test_exhaustive_n3_bruteforce():
    for W in P.exhaustive_n3():
        D, NX = oracle.fw_i32(W)
        dist, unique, first = P.brute_force(W.tolist())
        np.testing.assert_array_equal(D, np.array(dist), err_msg=str(W))
        bad, f = oracle.validate_walk(W, D, NX)
        assert bad == 0, (W, f)
        for i in range(3):
            for j in range(3):
                if unique[i][j] and dist[i][j] < INF:
                    assert NX[i, j] == first[i][j], (W, i, j)


@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (6, 3), (7, 4), (7, 5)])
def test_random_small_bruteforce(n, seed):
    for p, hi in [(0.3, 3), (0.6, 10), (1.0, 1000)]:
        W = rand_graph(n, seed, p, 1, hi)
        D, NX = oracle.fw_i32(W)
        dist, unique, first = P.brute_force(W.tolist())
        np.testing.assert_array_equal(D, np.array(dist))
        assert oracle.validate_walk(W, D, NX)[0] == 0
        for i in range(n):
            for j in range(n):
                if unique[i][j] and dist[i][j] < INF:
                    assert NX[i, j] == first[i][j]


@pytest.mark.parametrize("n,p,hi,seed", [(33, 0.1, 9, 11), (100, 0.5, 1000, 12),
                                         (257, 0.05, 100, 13), (300, 0.8, 10000, 14)])
def test_dijkstra_scipy_invariants(n, p, hi, seed):
    W = rand_graph(n, seed, p, 1, hi)
    fails, D, NX = check_all_pins_i32(W)
    assert not fails, fails
    absent = (W >= INF)
    S = P.scipy_dist(W, absent)
    Sd = np.where(np.isinf(S), INF, S).astype(np.int64)
    np.testing.assert_array_equal(D, Sd)


def test_closed_form_chain_cycle():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 40):
        w = rng.integers(1, 100, max(n - 1, 0))
        W, Dc, NXc = P.chain(n, w)
        D, NX = oracle.fw_i32(W)
        np.testing.assert_array_equal(D, Dc)
        np.testing.assert_array_equal(NX, NXc)
    for n in (2, 3, 17):
        w = rng.integers(1, 100, n)
        W, Dc, NXc = P.cycle(n, w)
        D, NX = oracle.fw_i32(W)
        np.testing.assert_array_equal(D, Dc)
        np.testing.assert_array_equal(NX, NXc)


def test_closed_form_complete_empty_star():
    n = 12
    W = np.full((n, n), 7, np.int64)
    np.fill_diagonal(W, 0)
    D, NX = oracle.fw_i32(W)
    np.testing.assert_array_equal(D, W)                     # 2w > w: direct edges stay
    np.testing.assert_array_equal(NX, np.tile(np.arange(n), (n, 1)))
    E = np.full((n, n), INF, np.int64)
    D, NX = oracle.fw_i32(E)
    exp = np.full((n, n), INF)
    np.fill_diagonal(exp, 0)
    np.testing.assert_array_equal(D, exp)
    np.testing.assert_array_equal(NX, np.where(np.eye(n, dtype=bool), np.arange(n)[:, None], -1))
    # star: spokes i -> 0 (a_i) and 0 -> j (b_j): D[i][j] = a_i + b_j
    a = np.arange(1, n) * 3
    b = np.arange(1, n) * 5 + 1
    S = np.full((n, n), INF, np.int64)
    np.fill_diagonal(S, 0)
    S[1:, 0] = a
    S[0, 1:] = b
    D, NX = oracle.fw_i32(S)
    for i in range(1, n):
        for j in range(1, n):
            if i != j:
                assert D[i, j] == a[i - 1] + b[j - 1] and NX[i, j] == 0


def test_input_normalisation():
    W = rand_graph(20, 5, 0.5, 1, 50).astype(np.int64)
    W2 = W.copy()
    W2[W2 >= INF] = np.iinfo(np.int32).max        # any value >= 2^30 is "absent"
    np.fill_diagonal(W2, 99)                       # self-loops are ignored
    D1, N1 = oracle.fw_i32(W)
    D2, N2 = oracle.fw_i32(W2)
    np.testing.assert_array_equal(D1, D2)
    np.testing.assert_array_equal(N1, N2)
    Wneg = W.copy()
    Wneg[0, 1] = -1
    with pytest.raises(ValueError):
        oracle.fw_i32(Wneg)


def test_float_oracles():
    # integer-valued float weights: every sum is exact, so f32/f64 == int32
    Wi = rand_graph(150, 21, 0.3, 1, 100)
    Wf = np.where(Wi >= INF, np.inf, Wi).astype(np.float32)
    Di, Ni = oracle.fw_i32(Wi)
    D32, N32 = oracle.fw_f32(Wf)
    D64, N64 = oracle.fw_f64(Wf)
    Dref = np.where(Di >= INF, np.inf, Di)
    np.testing.assert_array_equal(D32, Dref)
    np.testing.assert_array_equal(D64, Dref)
    np.testing.assert_array_equal(N32, Ni)
    np.testing.assert_array_equal(N64, Ni)
    # continuous weights: Dijkstra in float64, scipy, Bellman successor
    W = synth.graph_f32(200, 22, 0.4, 0.1, 10.0)
    D64, N64 = oracle.fw_f64(W)
    R = oracle.sssp_f64(W, np.arange(200))
    np.testing.assert_allclose(D64, R, rtol=1e-12)
    S = P.scipy_dist(np.where(np.isinf(W), 0, W), np.isinf(W))
    np.testing.assert_allclose(D64, S, rtol=1e-12)
    np.testing.assert_array_equal(N64, P.bellman_first_hop(W, D64))
    assert oracle.validate_walk(W, D64.astype(np.float32), N64, rtol=1e-6)[0] == 0
    D32, N32 = oracle.fw_f32(W)
    np.testing.assert_allclose(D32, D64, rtol=1e-6)
    with pytest.raises(ValueError):
        Wn = W.copy()
        Wn[1, 2] = np.nan
        oracle.fw_f64(Wn)


def test_unique_paths_next_hop_bellman():
    # complete graph, weights U[0.5, 1.5): unique shortest paths almost surely
    W = synth.graph_f32(160, 5, 1.0, 0.5, 1.5, g=99)
    D, NX = oracle.fw_f64(W)
    np.testing.assert_array_equal(NX, P.bellman_first_hop(W, D))


def test_thread_count_does_not_matter():
    W = rand_graph(200, 31, 0.2, 1, 20)             # many ties
    D1, N1 = oracle.fw_i32(W, nthreads=1)
    D8, N8 = oracle.fw_i32(W, nthreads=8)
    np.testing.assert_array_equal(D1, D8)
    np.testing.assert_array_equal(N1, N8)


def test_validator_rejects_broken_outputs():
    W = rand_graph(40, 41, 0.3, 1, 30)
    D, NX = oracle.fw_i32(W)
    reach = np.argwhere((D < INF) & ~np.eye(40, dtype=bool))
    i, j = reach[len(reach) // 2]
    D2 = D.copy(); D2[i, j] += 1
    assert oracle.validate_walk(W, D2, NX)[0] >= 1
    NX2 = NX.copy(); NX2[i, j] = i
    assert oracle.validate_walk(W, D, NX2)[0] >= 1
    NX3 = NX.copy(); NX3[0, 0] = -1
    assert oracle.validate_walk(W, D, NX3)[0] >= 1


def test_validator_f64_accepts_oracle_and_rejects_broken():
    W = synth.graph_f32(60, 41, 0.3, 0.1, 10.0).astype(np.float64)
    D, NX = oracle.fw_f64(W)
    assert oracle.validate_walk(W, D, NX, rtol=1e-12)[0] == 0
    D2 = D.copy()
    i, j = np.argwhere(np.isfinite(D2) & (D2 > 0))[5]
    D2[i, j] *= 1 + 1e-9                                   # a sum that no longer matches
    assert oracle.validate_walk(W, D2, NX, rtol=1e-12)[1][2] == 4
    N2 = NX.copy()
    N2[i, j] = i                                           # a walk that stays put
    assert oracle.validate_walk(W, D, N2, rtol=1e-12)[1][2] == 3
    D3 = D.copy()
    D3[0, 0] = 1.0
    assert oracle.validate_walk(W, D3, NX, rtol=1e-12)[1][2] == 1
