"""CPU model of successor tags (host logic, no GPU).

The three-launch int32 solve does not look up a successor when a phase-3
tile improves an entry (i, j) through vertex k: it stores a tag naming k
("the successor of (i, j) is that of (i, k)") and one pass after the last
round replaces every tag by the value of the entry it names, by pointer
jumping within the row.  The reading behind it: with exact (integer) sums,
the final distance is the shortest distance, so when a relaxation through k
gives (i, j) its final value, d(i, k) is already final (a later drop would
undercut d(i, j) through k), and a successor changes only with a strict
drop of its distance -- so the successor copied at that moment is the final
successor of (i, k).  This model runs blocked Floyd-Warshall (Section 2.3)
in plain Python with both bookkeepings on the same relaxation order and
checks that they give the same successors, bit for bit, on graphs full of
ties and zero weights, and long chains of tags; distances are checked
against the oracle.
"""
import numpy as np
import pytest

import oracle

INF = oracle.INF_I32
TAG = 1 << 30


def _blocked(W, bs, tags):
    """Blocked FW with a successor matrix; `tags` = "none" (eager copies),
    "phase3" (phase 3 stores tags, phases 1-2 copy whatever the entry holds,
    as the GPU path does) or "all" (every relaxation stores a tag)."""
    n = W.shape[0]
    D = np.minimum(W.astype(np.int64), INF)
    np.fill_diagonal(D, 0)
    NX = np.where(D < INF, np.arange(n)[None, :], -1).astype(np.int64)
    R = (n + bs - 1) // bs

    def relax(i, j, k, tag):
        if D[i, k] >= INF or D[k, j] >= INF:
            return
        s = D[i, k] + D[k, j]
        if s < D[i, j]:
            D[i, j] = s
            NX[i, j] = (TAG | k) if tag else NX[i, k]

    for K in range(R):
        blk = range(K * bs, min(n, K * bs + bs))
        rest = [v for v in range(n) if v not in blk]
        t12 = tags == "all"
        for k in blk:                                     # phase 1
            for i in blk:
                for j in blk:
                    relax(i, j, k, t12)
        for k in blk:                                     # phase 2
            for i in blk:
                for j in rest:
                    relax(i, j, k, t12)
            for i in rest:
                for j in blk:
                    relax(i, j, k, t12)
        for k in blk:                                     # phase 3
            for i in rest:
                for j in rest:
                    relax(i, j, k, tags != "none")
    return D, NX


def _resolve(NX):
    """Pointer jumping per row until no tag is left; returns the passes."""
    NX = NX.copy()
    passes = 0
    while True:
        t = (NX >= 0) & ((NX & TAG) != 0)
        if not t.any():
            return NX, passes
        assert passes < 40
        rows, cols = np.nonzero(t)
        NX[rows, cols] = NX[rows, NX[rows, cols] & (TAG - 1)]    # synchronous jump
        passes += 1


def _graph(rng, n, p, hi):
    W = rng.integers(0, hi + 1, size=(n, n)).astype(np.int64)
    W[rng.random((n, n)) >= p] = INF
    return W


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("tags", ["phase3", "all"])
def test_tags_give_eager_successors(seed, tags):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 30))
    bs = int(rng.choice([2, 3, 4, 8]))
    W = _graph(rng, n, float(rng.choice([0.15, 0.4, 0.9])), int(rng.choice([1, 3, 100])))
    De, Ne = _blocked(W, bs, "none")
    Dt, Nt = _blocked(W, bs, tags)
    Do, _ = oracle.fw_i32(W.astype(np.int32))
    np.testing.assert_array_equal(De, Do)
    np.testing.assert_array_equal(Dt, Do)
    Nr, _ = _resolve(Nt)
    np.testing.assert_array_equal(Nr, Ne)


def test_long_tag_chains_resolve_in_log_passes():
    """A directed path 0 -> 1 -> ... -> n-1 (and its reverse, heavier): the
    successor of (0, j) is named through a chain of about j tags, which
    pointer jumping resolves in about log2(n) passes."""
    n, bs = 64, 4
    W = np.full((n, n), INF, np.int64)
    for v in range(n - 1):
        W[v, v + 1] = 1
        W[v + 1, v] = 5
    De, Ne = _blocked(W, bs, "none")
    Dt, Nt = _blocked(W, bs, "all")
    np.testing.assert_array_equal(Dt, De)
    Nr, passes = _resolve(Nt)
    np.testing.assert_array_equal(Nr, Ne)
    np.testing.assert_array_equal(Ne[0, 1:], np.ones(n - 1))
    assert 4 <= passes <= 7


def test_tags_are_not_successors_themselves():
    """The tags carry intermediate vertices (the paper's path matrix P keeps
    one per entry too), not successors: read as successors without the
    resolution pass they differ, so the equality above is not vacuous."""
    rng = np.random.default_rng(3)
    W = _graph(rng, 24, 0.4, 3)
    _, Ne = _blocked(W, 4, "none")
    _, Nt = _blocked(W, 4, "phase3")
    t = (Nt >= 0) & ((Nt & TAG) != 0)
    assert t.sum() > 20
    raw = np.where(t, Nt & (TAG - 1), Nt)
    assert not np.array_equal(raw, Ne)


def _blocked_product(W, bs):
    """Blocked FW in the product form of the GPU kernels (phase 2 against the
    closed diagonal block and the band as it stood, phase 3 against both
    bands after phase 2; in each, the first k reaching the strict minimum),
    eager successors."""
    n = W.shape[0]
    D = np.minimum(W.astype(np.int64), INF)
    np.fill_diagonal(D, 0)
    NX = np.where(D < INF, np.arange(n)[None, :], -1).astype(np.int64)

    def product(rows, cols, ks, Acol, Brow, NXA):
        # C <- min(C, A (x) B), first k of the strict minimum; A/B/NXA frozen
        for i in rows:
            for j in cols:
                best, arg = D[i, j], -1
                for k in ks:
                    a, b = Acol[i][k], Brow[k][j]
                    if a < INF and b < INF and a + b < best:
                        best, arg = a + b, k
                if arg >= 0:
                    D[i, j] = best
                    NX[i, j] = NXA[i][arg]

    for K in range((n + bs - 1) // bs):
        blk = list(range(K * bs, min(n, K * bs + bs)))
        rest = [v for v in range(n) if v < blk[0] or v > blk[-1]]
        for k in blk:                                      # phase 1, in place
            for i in blk:
                for j in blk:
                    if D[i, k] < INF and D[k, j] < INF and D[i, k] + D[k, j] < D[i, j]:
                        D[i, j] = D[i, k] + D[k, j]
                        NX[i, j] = NX[i, k]
        Dc, Nc = D.copy(), NX.copy()
        product(blk, rest, blk, Dc, Dc, Nc)                # row band: A = closed block, B = old band
        product(rest, blk, blk, Dc, Dc, Nc)                # column band: A = old band, B = closed block
        Dc, Nc = D.copy(), NX.copy()
        product(rest, rest, blk, Dc, Dc, Nc)               # phase 3: both bands after phase 2
    return D, NX


def _walks_end(NX, n):
    for i in range(n):
        for j in range(n):
            if NX[i, j] < 0:
                continue
            v, steps = i, 0
            while v != j:
                v = NX[v, j]
                steps += 1
                if steps > n:
                    return False
    return True


def test_product_form_walks_end_without_zero_cycles():
    """Positive cycles only (zero-weight edges allowed on a DAG): the
    product form's successor walks all reach their destination."""
    rng = np.random.default_rng(5)
    n = 40
    W = _graph(rng, n, 0.15, 2)
    lower = np.tril(np.ones((n, n), bool), -1)
    W[lower & (W == 0)] = 1                            # zero weights only on edges i -> j, i < j
    D, NX = _blocked_product(W, 8)
    Do, _ = oracle.fw_i32(W.astype(np.int32))
    np.testing.assert_array_equal(D, Do)
    assert _walks_end(NX, n)


def test_product_form_can_loop_on_zero_cycles():
    """With zero-weight cycles the distances stay exact, but a successor walk
    can circle inside a zero-weight cycle: phase 3 takes both bands after
    phase 2, so a path i -> k and a path k -> j may share a vertex x, and
    the zero-weight cycle through x and k then ties with the shortcut
    through x.  The plain triple loop never does this (its operands at step k
    use intermediates below k only)."""
    rng = np.random.default_rng(7)
    found = False
    for _ in range(20):
        n = 36
        W = _graph(rng, n, 0.08, 1)                    # sparse, weights 0 or 1: zero cycles
        D, NX = _blocked_product(W, 6)
        Do, NXo = oracle.fw_i32(W.astype(np.int32))
        np.testing.assert_array_equal(D, Do)
        assert _walks_end(NXo, n)
        if not _walks_end(NX, n):
            found = True
            break
    assert found
