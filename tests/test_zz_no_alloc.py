"""The allocation-free batched solve (fw_solve_batched_static) against the
allocating one (fw_solve_batched_*): the same bits on two calls in a row,
the second with a smaller batch, for each element type, one workgroup per
graph and team schedules; its device error word is reported by fw_check;
requests beyond its fixed scratch are refused before anything is enqueued."""
import numpy as np
import pytest

from tests.gpu_helpers import log
from tests.test_gpu_batched import make_batch

pytestmark = pytest.mark.gpu


def run(arena, offs, sizes, n_max, static, team, next_hop=True):
    import torch
    import paper_2403_18619_amd as fw
    D = torch.from_numpy(arena.copy()).cuda()
    NX = torch.full((arena.size,), -7, dtype=torch.int32, device="cuda") if next_hop else None
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    fw.solve_batched_(D, NX, off, sz, n_max, team=team, static=static)
    fw.check()
    return D.cpu().numpy(), (NX.cpu().numpy() if next_hop else None)


def batch(sizes, dtype, seed):
    graphs, offs, arena = make_batch(sizes, "i32" if dtype == "i32" else "f32", seed)
    if dtype == "f64":
        arena = arena.astype(np.float64)
    return offs, arena


FIRST = [300, 1, 0, 17, 128, 129, 256, 64, 400, 200, 33, 5, 255, 384, 100]
SECOND = [150, 3, 64, 0, 130, 90]          # fewer and smaller graphs


@pytest.mark.parametrize("team", [1, 4])
@pytest.mark.parametrize("dtype", ["i32", "f32", "f64"])
def test_static_matches_allocating_twice(dtype, team):
    for call, sizes in enumerate((FIRST, SECOND)):
        log(f"case no_alloc {dtype} team={team} call={call} graphs={len(sizes)} n_max={max(sizes)}")
        offs, arena = batch(sizes, dtype, 40 + call)
        n_max = max(sizes)
        Ds, Ns = run(arena, offs, sizes, n_max, static=True, team=team)
        Da, Na = run(arena, offs, sizes, n_max, static=False, team=team)
        view = np.uint64 if dtype == "f64" else np.uint32
        np.testing.assert_array_equal(Ds.view(view), Da.view(view), err_msg=f"call {call}")
        np.testing.assert_array_equal(Ns, Na, err_msg=f"call {call}")
        Dd, _ = run(arena, offs, sizes, n_max, static=True, team=team, next_hop=False)
        Dad, _ = run(arena, offs, sizes, n_max, static=False, team=team, next_hop=False)
        np.testing.assert_array_equal(Dd.view(view), Dad.view(view), err_msg=f"call {call}, distances only")


def test_static_reports_device_errors_and_refuses_oversize():
    import torch
    import paper_2403_18619_amd as fw
    log("case no_alloc errors")
    sizes = [40, 20]
    offs, arena = batch(sizes, "f32", 50)
    D = torch.from_numpy(arena.copy()).cuda()
    off = torch.from_numpy(offs).cuda()
    bad = torch.tensor([40, 41], dtype=torch.int32, device="cuda")     # 41 > n_max
    fw.solve_batched_(D, None, off, bad, 40, static=True)
    with pytest.raises(fw.FwError) as e:
        fw.check()
    assert e.value.status == fw.FW_ERR_INVALID_ARG
    fw.check()                                      # cleared
    # a request whose order arrays and team flags exceed the fixed scratch
    big = torch.zeros(65535, dtype=torch.int32, device="cuda")
    boff = torch.zeros(65535, dtype=torch.int64, device="cuda")
    before = D.clone()
    with pytest.raises(fw.FwError) as e:
        fw.solve_batched_(D, None, boff, big, 65536, team=1000, static=True)
    assert e.value.status == fw.FW_ERR_UNSUPPORTED
    assert "scratch" in fw.last_error()
    torch.cuda.synchronize()
    assert torch.equal(D, before)                   # nothing was enqueued
    fw.check()
