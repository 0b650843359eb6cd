"""Batched solves (fw_solve_batched_*): every graph of the batch gets the same
bits as a single solve with block size 128, distances match the oracle, bad
sizes are reported, and the call replays correctly from a captured HIP graph."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import INF, assert_close_f32, assert_walks, gpu_solve, log

pytestmark = pytest.mark.gpu


def make_batch(sizes, dtype, seed):
    """Pack graphs into one arena: graph g = recipe graph of size sizes[g]."""
    graphs = []
    for g, n in enumerate(sizes):
        if dtype == "i32":
            graphs.append(synth.graph_i32(int(n), seed, 0.3, 1, 50, g=g + 1))
        else:
            graphs.append(synth.graph_f32(int(n), seed, 0.3, 0.1, 10.0, g=g + 1))
    offs = np.zeros(len(sizes), np.int64)
    tot = 0
    for g, n in enumerate(sizes):
        offs[g] = tot
        tot += int(n) * int(n)
    arena = np.zeros(max(tot, 1), np.int32 if dtype == "i32" else np.float32)
    for g, n in enumerate(sizes):
        arena[offs[g]:offs[g] + n * n] = graphs[g].reshape(-1)
    return graphs, offs, arena


def run_batched(arena, offs, sizes, n_max, next_hop=True, flags=0, team=0):
    import torch
    import paper_2403_18619_amd as fw
    D = torch.from_numpy(arena.copy()).cuda()
    NX = torch.empty(arena.size, dtype=torch.int32, device="cuda") if next_hop else None
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    fw.solve_batched_(D, NX, off, sz, n_max, flags=flags, team=team)
    fw.check()
    return D.cpu().numpy(), (NX.cpu().numpy() if next_hop else None)


@pytest.mark.parametrize("team", [1, 0, 3, 1000])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
@pytest.mark.parametrize("next_hop", [True, False])
def test_batched_matches_single_solves(dtype, next_hop, team):
    """Every graph bit-equal to single solves with both schedules, for one
    workgroup per graph (team 1), the automatic limit and team schedules."""
    log(f"case batched vs single {dtype} next={next_hop} team={team}")
    sizes = [1, 0, 2, 17, 64, 127, 128, 129, 200, 255, 256, 300, 33, 5, 700, 513, 384]
    graphs, offs, arena = make_batch(sizes, dtype, 11)
    D, NX = run_batched(arena, offs, sizes, 700, next_hop, team=team)
    import paper_2403_18619_amd as fw
    for g, n in enumerate(sizes):
        if n == 0:
            continue
        Dg = D[offs[g]:offs[g] + n * n].reshape(n, n)
        for sched in (fw.SCHED_THREE_LAUNCH, fw.SCHED_AUTO):
            Ds, Ns = gpu_solve(graphs[g], next_hop=next_hop, block=128, schedule=sched)
            msg = f"graph {g} n={n} schedule {sched}"
            np.testing.assert_array_equal(Dg.view(np.uint32), Ds.view(np.uint32), err_msg=msg)
            if next_hop:
                np.testing.assert_array_equal(NX[offs[g]:offs[g] + n * n].reshape(n, n), Ns, err_msg=msg)


@pytest.mark.parametrize("team", [2, 1000])
def test_batched_team_repeatable_f32(team):
    """Team schedules read other workgroups' tiles through flags: repeated
    float32 runs stay bit-equal (a stale read would change low bits)."""
    log(f"case batched team repeat team={team}")
    sizes = [600, 450, 300, 260, 1000]
    graphs, offs, arena = make_batch(sizes, "f32", 21)
    D0, N0 = run_batched(arena, offs, sizes, 1000, team=1)
    for rep in range(4):
        D, NX = run_batched(arena, offs, sizes, 1000, team=team)
        np.testing.assert_array_equal(D.view(np.uint32), D0.view(np.uint32), err_msg=f"run {rep}")
        np.testing.assert_array_equal(NX, N0, err_msg=f"run {rep}")


def test_batched_team_timeout_is_reported():
    log("case batched team timeout")
    import paper_2403_18619_amd as fw
    sizes = [700, 500, 64]
    graphs, offs, arena = make_batch(sizes, "i32", 22)
    with pytest.raises(fw.FwError) as e:
        run_batched(arena, offs, sizes, 700, flags=fw.FLAG_TEST_TIMEOUT, team=16)
    assert e.value.status == fw.FW_ERR_TIMEOUT
    D, _ = run_batched(arena, offs, sizes, 700, team=16)         # the next solve is unaffected
    for g, n in enumerate(sizes):
        Dr, _ = oracle.fw_i32(graphs[g], next_hop=False)
        np.testing.assert_array_equal(D[offs[g]:offs[g] + n * n].reshape(n, n), Dr)


def test_autotuners_restore_input_and_agree():
    """The tuners leave dist as it was, return one of their candidates, and the
    automatic choice afterwards gives the same bits as before."""
    log("case autotuners")
    import torch
    import paper_2403_18619_amd as fw
    sizes = [300, 520, 130, 90]
    graphs, offs, arena = make_batch(sizes, "f32", 23)
    D = torch.from_numpy(arena.copy()).cuda()
    NX = torch.empty(arena.size, dtype=torch.int32, device="cuda")
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    team, ms = fw.tune_batched_(D, NX, off, sz, 520, reps=1)
    assert team in (1, 2, 4, 8, 16, 25) and ms > 0
    assert np.array_equal(D.cpu().numpy().view(np.uint32), arena.view(np.uint32))
    Dt, Nt = run_batched(arena, offs, sizes, 520, team=0)
    D1, N1 = run_batched(arena, offs, sizes, 520, team=1)
    np.testing.assert_array_equal(Dt.view(np.uint32), D1.view(np.uint32))
    np.testing.assert_array_equal(Nt, N1)
    W = synth.graph_f32(700, 24, 1.0, 0.0, 1.0)
    Wd = torch.from_numpy(W).cuda()
    Nd = torch.empty_like(Wd, dtype=torch.int32)
    block, sched, ms = fw.tune_solve_(Wd, Nd, reps=1)
    assert (block, sched) in ((32, 1), (64, 1), (128, 1), (128, 2)) and ms > 0
    assert np.array_equal(Wd.cpu().numpy().view(np.uint32), W.view(np.uint32))
    Da, Na = gpu_solve(W)                                         # automatic: the tuned choice
    Db, Nb = gpu_solve(W, block=block, schedule=sched)
    np.testing.assert_array_equal(Da.view(np.uint32), Db.view(np.uint32))
    np.testing.assert_array_equal(Na, Nb)


def test_batched_recipe_against_oracle():
    """A slice of the batched recipe (n ~ U{16..256}, edge prob 0.3, float32
    U[0.1,10)): every graph against the float64 oracle, walks valid."""
    log("case batched recipe vs oracle")
    sizes = synth.batch_sizes()[:96]
    graphs = [synth.batch_graph_f32(int(n), g) for g, n in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum([int(n) * int(n) for n in sizes])[:-1]]).astype(np.int64)
    arena = np.concatenate([w.reshape(-1) for w in graphs])
    D, NX = run_batched(arena, offs, sizes, 256)
    for g, n in enumerate(sizes):
        n = int(n)
        Dg = D[offs[g]:offs[g] + n * n].reshape(n, n)
        Ng = NX[offs[g]:offs[g] + n * n].reshape(n, n)
        D64, _ = oracle.fw_f64(graphs[g], next_hop=False)
        assert_close_f32(Dg, D64)
        assert_walks(graphs[g], Dg, Ng)


def test_batched_int_exact_and_eager_equal():
    log("case batched int exact + eager")
    import paper_2403_18619_amd as fw
    sizes = [40, 180, 250, 7, 129]
    graphs, offs, arena = make_batch(sizes, "i32", 12)
    D, NX = run_batched(arena, offs, sizes, 256)
    D2, NX2 = run_batched(arena, offs, sizes, 256, flags=fw.FLAG_EAGER_ARGMIN)
    np.testing.assert_array_equal(D, D2)
    np.testing.assert_array_equal(NX, NX2)
    for g, n in enumerate(sizes):
        Dr, _ = oracle.fw_i32(graphs[g], next_hop=False)
        np.testing.assert_array_equal(D[offs[g]:offs[g] + n * n].reshape(n, n), Dr)


def test_batched_size_beyond_bound_is_reported():
    log("case batched bad size")
    import paper_2403_18619_amd as fw
    sizes = [10, 20]
    graphs, offs, arena = make_batch(sizes, "i32", 13)
    with pytest.raises(fw.FwError) as e:
        run_batched(arena, offs, sizes, 15)
    assert e.value.status == fw.FW_ERR_INVALID_ARG
    fw.check()


def test_batched_hip_graph_replays():
    """Capture input restore + batched solve once, replay it with eager work in
    between; every replay must reproduce the eager result."""
    log("case batched hip graph")
    import torch
    import paper_2403_18619_amd as fw
    sizes = [int(x) for x in synth.batch_sizes(count=64)]
    graphs = [synth.batch_graph_f32(n, g) for g, n in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    W0 = torch.from_numpy(np.concatenate([w.reshape(-1) for w in graphs])).cuda()
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    D = torch.empty_like(W0)
    NX = torch.empty(W0.numel(), dtype=torch.int32, device="cuda")
    D.copy_(W0)
    fw.solve_batched_(D, NX, off, sz, 256)            # warm-up: workspace allocated
    torch.cuda.synchronize()
    fw.check()
    ref_d, ref_n = D.clone(), NX.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        D.copy_(W0)
        fw.solve_batched_(D, NX, off, sz, 256)
    for rep in range(3):
        D.fill_(0.0)
        NX.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(D.view(torch.int32), ref_d.view(torch.int32)), rep
        assert torch.equal(NX, ref_n), rep
    fw.check()
