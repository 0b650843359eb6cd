"""float64 distances (fw_solve_*_f64): against the float64 oracle, across
block sizes, schedules, successor variants and the batched solve.

Tolerance: the GPU adds sub-path sums in blocked (tree) order, the oracle in
the triple loop's order; both round every sum to double, so a distance over
h hops differs by at most about (h - 1) 2^-53 relative.  1e-12 covers paths of
thousands of hops.  With integer-valued weights every sum is exact and the
distances must be bit-equal.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import gpu_solve, log

pytestmark = pytest.mark.gpu
RTOL = 1e-12


def graph64(n, seed, p, a, b, integer=False):
    W = synth.graph_f32(n, seed, p, a, b).astype(np.float64)
    if integer:
        W = np.where(np.isfinite(W), np.floor(W), W)
        np.fill_diagonal(W, 0.0)
    return W


def check_against_oracle(W, Dg, NXg, exact):
    Do, NXo = oracle.fw_f64(W)
    assert (np.isinf(Dg) == np.isinf(Do)).all()
    fin = np.isfinite(Do)
    if exact:
        np.testing.assert_array_equal(Dg, Do)
    else:
        err = np.abs(Dg[fin] - Do[fin])
        assert (err <= RTOL * np.abs(Do[fin])).all(), f"worst rel {np.max(err / np.maximum(Do[fin], 1e-300)):.3g}"
    if NXg is not None:
        bad, first = oracle.validate_walk(W, Dg, NXg, rtol=RTOL)
        assert bad == 0, f"{bad} bad walks, first {first}"
        if not exact:                           # continuous weights: successors unique up to near-ties
            diff = np.argwhere(NXg != NXo)
            for i, j in diff:
                h = NXg[i, j]
                alt = W[i, h] + Do[h, j]
                assert abs(alt - Do[i, j]) <= RTOL * abs(Do[i, j]), (i, j, h)


@pytest.mark.parametrize("n", [1, 2, 100, 129, 300, 1000])
@pytest.mark.parametrize("recipe", ["continuous", "integer", "sparse"])
def test_f64_against_oracle(n, recipe):
    log(f"case f64 {recipe} n={n}")
    if recipe == "continuous":
        W = graph64(n, 500 + n, 1.0, 0.0, 1.0)
    elif recipe == "integer":
        W = graph64(n, 600 + n, 0.5, 1.0, 50.0, integer=True)
    else:
        W = graph64(n, 700 + n, 0.05, 0.1, 10.0)
    Dg, NXg = gpu_solve(W)
    check_against_oracle(W, Dg, NXg, exact=recipe == "integer")


@pytest.mark.parametrize("n", [257, 700])
def test_f64_block_sizes_schedules_and_variants(n):
    """Block 32/64/128 with three launches and the persistent schedule: bit-equal
    distances on integer weights; at block 128 every schedule and both
    successor variants give the same bits on continuous weights."""
    log(f"case f64 schedules n={n}")
    import paper_2403_18619_amd as fw
    Wi = graph64(n, 800 + n, 0.4, 1.0, 30.0, integer=True)
    ref, _ = gpu_solve(Wi, block=128, schedule=fw.SCHED_THREE_LAUNCH)
    for block, sched in ((32, 1), (64, 1), (128, 2)):
        D, NX = gpu_solve(Wi, block=block, schedule=sched)
        np.testing.assert_array_equal(D, ref)
        assert oracle.validate_walk(Wi, D, NX, rtol=RTOL)[0] == 0
    Wc = graph64(n, 900 + n, 0.6, 0.0, 1.0)
    D1, N1 = gpu_solve(Wc, block=128, schedule=fw.SCHED_THREE_LAUNCH)
    for sched, flags in ((fw.SCHED_PERSISTENT, 0), (fw.SCHED_THREE_LAUNCH, fw.FLAG_EAGER_ARGMIN),
                         (fw.SCHED_PERSISTENT, fw.FLAG_EAGER_ARGMIN)):
        D2, N2 = gpu_solve(Wc, block=128, schedule=sched, flags=flags)
        np.testing.assert_array_equal(D2.view(np.uint64), D1.view(np.uint64))
        np.testing.assert_array_equal(N2, N1)
    Dd, _ = gpu_solve(Wc, next_hop=False, block=128, schedule=fw.SCHED_PERSISTENT)
    np.testing.assert_array_equal(Dd.view(np.uint64), D1.view(np.uint64))
    check_against_oracle(Wc, D1, N1, exact=False)


@pytest.mark.parametrize("team", [1, 0, 1000])
def test_f64_batched_matches_single(team):
    log(f"case f64 batched team={team}")
    import torch
    import paper_2403_18619_amd as fw
    sizes = [300, 1, 0, 129, 17, 600, 256]
    graphs = [graph64(n, 1000 + g, 0.3, 0.1, 10.0) for g, n in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    arena = np.concatenate([w.reshape(-1) for w in graphs])
    D = torch.from_numpy(arena).cuda()
    NX = torch.empty(arena.size, dtype=torch.int32, device="cuda")
    fw.solve_batched_(D, NX, torch.from_numpy(offs).cuda(),
                      torch.from_numpy(np.asarray(sizes, np.int32)).cuda(), 600, team=team)
    fw.check()
    Dh, Nh = D.cpu().numpy(), NX.cpu().numpy()
    for g, n in enumerate(sizes):
        if n == 0:
            continue
        Ds, Ns = gpu_solve(graphs[g], block=128, schedule=fw.SCHED_THREE_LAUNCH)
        np.testing.assert_array_equal(Dh[offs[g]:offs[g] + n * n].reshape(n, n).view(np.uint64), Ds.view(np.uint64))
        np.testing.assert_array_equal(Nh[offs[g]:offs[g] + n * n].reshape(n, n), Ns)


def test_f64_dense_2048_and_padded_rows():
    log("case f64 dense 2048 + ld padding")
    W = graph64(2048, 1101, 1.0, 0.0, 1.0)
    Dg, NXg = gpu_solve(W)
    check_against_oracle(W, Dg, NXg, exact=False)
    W = graph64(333, 1102, 0.3, 0.1, 10.0)
    Dp, Np = gpu_solve(W, ld=341)
    Dq, Nq = gpu_solve(W)
    np.testing.assert_array_equal(Dp.view(np.uint64), Dq.view(np.uint64))
    np.testing.assert_array_equal(Np, Nq)
