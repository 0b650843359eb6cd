"""Gradient pass (fw_backward_f32 / fw_backward_batched_f32) against the
reference gradient of the oracle (oracle.grad_ref, pinned by finite
differences in test_oracle_grad.py), on the successor matrix the GPU solve
returned, so that both walk the same paths.

Tolerance: every gradient entry is a float32 sum of upstream values, first
into subtree sums (at most n levels, at most n children per vertex), then over
at most n destinations.  Each addition rounds with relative error 2^-24 of a
partial sum bounded by the sum of |upstream| over the entry's contributions
(ref_abs), so |got - ref| <= 3 n 2^-24 ref_abs.  Entries with no contribution
must be exactly 0.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import gpu_solve, log

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def assert_grad_close(got, G, NX):
    ref = oracle.grad_ref(G, NX)
    ref_abs = oracle.grad_abs_ref(G, NX)
    n = NX.shape[0]
    tol = 3 * n * U * ref_abs
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > tol
    if bad.any():
        u, v = np.argwhere(bad)[0]
        raise AssertionError(f"{int(bad.sum())} entries off; first ({u},{v}): got {got[u, v]!r} "
                             f"ref {ref[u, v]!r} tol {tol[u, v]!r}")
    assert not got[ref_abs == 0].any()


def gpu_backward(G, NX):
    import torch
    import paper_2403_18619_amd as fw
    Gd = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    Nd = torch.from_numpy(np.ascontiguousarray(NX)).cuda()
    dW = torch.full_like(Gd, 7.0)                  # overwritten, not accumulated into
    fw.backward_(Gd, Nd, dW)
    fw.check()
    return dW.cpu().numpy()


RECIPES = {
    "complete": lambda n, s: synth.graph_f32(n, s, 1.0, 0.5, 1.5),      # the fwd+bwd recipe
    "sparse": lambda n, s: synth.graph_f32(n, s, 0.3, 0.1, 10.0),
    "very_sparse": lambda n, s: synth.graph_f32(n, s, 4.0 / max(n, 1), 0.1, 10.0),
}


@pytest.mark.parametrize("recipe", sorted(RECIPES))
@pytest.mark.parametrize("n", [2, 17, 128, 129, 300, 1000])
def test_backward_matches_reference(recipe, n):
    log(f"case backward {recipe} n={n}")
    W = RECIPES[recipe](n, 700 + n)
    G = synth.normal_f32(n, n, 800 + n)
    _, NX = gpu_solve(W)
    assert_grad_close(gpu_backward(G, NX), G, NX)


def test_backward_padded_rows_and_large_n_scratch_path():
    """ld > n; the three kernel forms: one wave per destination (n <= 1024),
    one workgroup with LDS arrays (n <= 4096), one workgroup with global
    arrays (above)."""
    log("case backward ld padding + n=2000 + n=4500")
    import torch
    import paper_2403_18619_amd as fw
    for n, ld in ((300, 333), (2000, 2003), (4500, 4500)):
        W = synth.graph_f32(n, 901, 0.002 if n > 1000 else 0.3, 0.1, 10.0)
        G = synth.normal_f32(n, n, 902)
        _, NX = gpu_solve(W)
        Gd = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
        Nd = torch.zeros((n, ld), dtype=torch.int32, device="cuda")
        dW = torch.full((n, ld), 5.0, dtype=torch.float32, device="cuda")
        Gd[:, :n].copy_(torch.from_numpy(G))
        Nd[:, :n].copy_(torch.from_numpy(NX))
        fw.backward_(Gd[:, :n], Nd[:, :n], dW[:, :n])
        fw.check()
        out = dW.cpu().numpy()
        assert_grad_close(out[:, :n], G, NX)
        assert (out[:, n:] == 5.0).all()             # padding untouched


def test_autograd_function():
    """FloydWarshall.apply: D equals a plain solve and W.grad the gradient pass."""
    log("case autograd")
    import torch
    import paper_2403_18619_amd as fw
    n = 200
    W = synth.graph_f32(n, 911, 0.3, 0.1, 10.0)
    G = synth.normal_f32(n, n, 912)
    Wt = torch.from_numpy(W).cuda().requires_grad_(True)
    D, NX = fw.shortest_paths(Wt)
    Dref, NXref = gpu_solve(W)
    np.testing.assert_array_equal(D.detach().cpu().numpy().view(np.uint32), Dref.view(np.uint32))
    np.testing.assert_array_equal(NX.cpu().numpy(), NXref)
    Gt = torch.from_numpy(G).cuda()
    loss = (torch.where(torch.isfinite(D), D, torch.zeros_like(D)) * Gt).sum()
    loss.backward()
    assert_grad_close(Wt.grad.cpu().numpy(), G, NXref)
    assert NX.requires_grad is False


def test_backward_batched_against_reference():
    """A slice of the fwd+bwd recipe (complete graphs, n ~ U{64..1024},
    weights U[0.5,1.5), N(0,1) upstream) plus small and empty graphs."""
    log("case backward batched")
    import torch
    import paper_2403_18619_amd as fw
    sizes = [int(x) for x in synth.fwdbwd_sizes()[:10]] + [0, 1, 2, 65]
    graphs = [synth.fwdbwd_graph_f32(n, g) if n else np.zeros((0, 0), np.float32) for g, n in enumerate(sizes)]
    ups = [synth.fwdbwd_upstream(n, g) if n else np.zeros((0, 0), np.float32) for g, n in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    n_max = max(sizes)
    D = torch.from_numpy(np.concatenate([w.reshape(-1) for w in graphs])).cuda()
    G = torch.from_numpy(np.concatenate([u.reshape(-1) for u in ups])).cuda()
    NX = torch.empty(D.numel(), dtype=torch.int32, device="cuda")
    dW = torch.full_like(D, 3.0)
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    fw.solve_batched_(D, NX, off, sz, n_max)
    fw.backward_batched_(G, NX, dW, off, sz, n_max)
    fw.check()
    NXh, dWh = NX.cpu().numpy(), dW.cpu().numpy()
    for g, n in enumerate(sizes):
        if n == 0:
            continue
        sl = slice(offs[g], offs[g] + n * n)
        assert_grad_close(dWh[sl].reshape(n, n), ups[g], NXh[sl].reshape(n, n))


def test_backward_batched_hip_graph_replays():
    log("case backward batched hip graph")
    import torch
    import paper_2403_18619_amd as fw
    sizes = [100, 37, 256, 5]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])[:-1]]).astype(np.int64)
    W = np.concatenate([synth.graph_f32(n, 920 + g, 0.3, 0.1, 10.0).reshape(-1) for g, n in enumerate(sizes)])
    Gh = np.concatenate([synth.normal_f32(n, n, 930 + g).reshape(-1) for g, n in enumerate(sizes)])
    D = torch.from_numpy(W).cuda()
    NX = torch.empty(D.numel(), dtype=torch.int32, device="cuda")
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    fw.solve_batched_(D, NX, off, sz, 256)
    G = torch.from_numpy(Gh).cuda()
    dW = torch.empty_like(G)
    fw.backward_batched_(G, NX, dW, off, sz, 256)
    torch.cuda.synchronize()
    fw.check()
    ref = dW.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fw.backward_batched_(G, NX, dW, off, sz, 256)
    NXh = NX.cpu().numpy()
    for rep in range(3):
        dW.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = dW.cpu().numpy()
        for g, n in enumerate(sizes):
            sl = slice(offs[g], offs[g] + n * n)
            assert_grad_close(got[sl].reshape(n, n), Gh[sl].reshape(n, n), NXh[sl].reshape(n, n))
        # run-to-run differences are rounding only
        np.testing.assert_allclose(got, ref.cpu().numpy(), rtol=1e-4, atol=1e-4)
    fw.check()


def test_backward_malformed_successors_end():
    """Out-of-range successors count as no path and a successor cycle adds
    nothing: the kernel ends and the rest of the column is still right."""
    log("case backward malformed")
    n = 6
    NX = np.tile(np.arange(n, dtype=np.int32), (n, 1))     # direct edge to every destination
    G = synth.normal_f32(n, n, 940)
    # destination 0: 1 -> 2 -> 1 is a cycle, 3 -> 99 leaves the range, 4 -> 5 -> 0 is valid
    NX[1, 0], NX[2, 0], NX[3, 0], NX[4, 0], NX[5, 0] = 2, 1, 99, 5, 0
    got = gpu_backward(G, NX)
    want = np.zeros((n, n), np.float64)
    for i in range(n):
        for j in range(1, n):
            if i != j:
                want[i, j] += G[i, j]                       # direct edges
    want[4, 5] += G[4, 0]
    want[5, 0] += G[4, 0] + G[5, 0]
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-6)
