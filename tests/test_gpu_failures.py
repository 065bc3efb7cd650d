"""Failure handling forced from the host: corrupted caller-owned state is
reported by lb_check (LB_ESTATE) without faulting, invalid schedules and
misuse of views are rejected before anything is enqueued, and a context
recovers from a restored checkpoint bit for bit."""
import ctypes

import pytest
import torch

import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb

pytestmark = pytest.mark.gpu

CFG = dict(nx=12, ny=10, nz=8, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5, gamma_odd=0.0,
           gamma_even=0.0, seed=9)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_nan_and_negative_density_reported(storage):
    lat = lbf.Lattice(**CFG, storage=storage, init="thermal")
    lat.step(2)
    assert lat.check()[0] == 0
    snap = lat.state.clone()
    # a NaN population at one site (even t: plane i at site r holds n_i(r))
    lat.state[5, 3, 4, 6] = float("nan")
    nb, _ = lat.check()
    assert nb == 1
    rc = lb.lib().lb_check(lat._ctx, None, None)
    assert rc == lb.LB_ESTATE
    # rho <= 0 at another site: d_i = -1 (n_i = 0) for every population
    lat.state.copy_(snap)
    lat.state[:, 1, 2, 3] = -1.0
    nb, _ = lat.check()
    assert nb == 1
    # restore the snapshot: the context continues as if nothing happened
    lat.state.copy_(snap)
    lat.step(3)
    ref = lbf.Lattice(**CFG, storage=storage, init="thermal")
    ref.step(5)
    assert torch.equal(lat.state, ref.state)
    assert lat.check()[0] == 0


def test_invalid_schedules_rejected():
    lat = lbf.Lattice(**CFG, init="rest")
    before = lat.schedule()
    for bad in [dict(block=96), dict(order=3), dict(graph_chunk=3), dict(graph_chunk=0), dict(xcd_remap=65), dict(xcd_remap=-1),
                dict(tiling=(0, 5)), dict(resident=2), dict(resident=-1), dict(group_mb=-1),
                dict(group_mb=(1 << 20) + 1), dict(fused=2), dict(fused=-1)]:
        args = dict(block=256, order=0, xcd_remap=0, graph_chunk=16, tiling=0)
        args.update(bad)
        with pytest.raises(lb.LBError) as ei:
            lat.set_schedule(**args)
        assert ei.value.code == lb.LB_EINVAL
    assert lat.schedule() == before
    with pytest.raises(lb.LBError):
        lat.step(-1)


def test_views_cannot_step_and_batches_need_views():
    ens = lbf.Ensemble([dict(nx=4, ny=4, nz=4, kT=1e-4, seed=1), dict(nx=5, ny=3, nz=2, kT=1e-4, seed=2)])
    v = ens.view(1)
    L = lb.lib()
    assert L.lb_step(v._ctx, 1) == lb.LB_EINVAL
    assert L.lb_batch_step(v._ctx, 1) == lb.LB_EINVAL
    out = torch.empty((4, 4, 4, 4), device="cuda")
    assert L.lb_moments(ens._ctx, ctypes.c_void_p(out.data_ptr())) == lb.LB_EINVAL
    sub = ctypes.c_void_p()
    assert L.lb_batch_view(v._ctx, 0, ctypes.byref(sub)) == lb.LB_EINVAL
    assert L.lb_batch_view(ens._ctx, 2, ctypes.byref(sub)) == lb.LB_EINVAL
    ens.step(3)
    assert v.t == 3
    assert v.check()[0] == 0
    ens.close()


def test_init_argument_errors_on_device():
    p = lb.make_params(4, 4, 4)
    buf = torch.empty(19 * 64 + 64, device="cuda")
    ctx = ctypes.c_void_p()
    L = lb.lib()
    # misaligned state pointer (4 bytes past a 256-byte boundary)
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(buf.data_ptr() + 4), None, 0, None, 0,
                     ctypes.byref(ctx)) == lb.LB_EINVAL
    # fields missing for the FIELDS initial state
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(buf.data_ptr()), None, 2, None, 0,
                     ctypes.byref(ctx)) == lb.LB_EINVAL
    assert ctx.value is None


def test_bf16_without_noise_warns():
    with pytest.warns(UserWarning, match="bf16 storage without thermal noise is biased"):
        lat = lbf.Lattice(nx=8, ny=8, nz=8, storage="bf16", kT=0.0, init="rest")
    assert "warning: bf16" in lb.lib().lb_last_error().decode()
    lat.close()


def test_autotune_without_room_for_its_scratch_copy():
    """The autotuner needs a scratch copy of the state: with less free device
    memory than that it returns LB_EUNSUPPORTED and changes nothing."""
    lat = lbf.Lattice(nx=512, ny=512, nz=256, storage="f32", kT=1e-4, seed=3, init="thermal")  # 5.1 GB
    lat.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0)
    before = lat.schedule()
    state = lat.state.clone()
    torch.cuda.synchronize()
    free = torch.cuda.mem_get_info()[0]
    filler = torch.empty(max(free - (2 << 30), 0), dtype=torch.uint8, device="cuda")  # leave 2 GiB free
    try:
        with pytest.raises(lb.LBError) as ei:
            lat.autotune(steps=2)
        assert ei.value.code == lb.LB_EUNSUPPORTED
        assert "scratch copy" in str(ei.value)
    finally:
        del filler
        torch.cuda.empty_cache()
    assert lat.schedule() == before and lat.t == 0
    assert torch.equal(lat.state, state)
    lat.close()
