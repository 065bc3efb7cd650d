"""lb_step_noalloc, the step entry point that allocates nothing, against the
context-based entry points it mirrors (lb_batch_step, lb_step): the same
bits, on two calls in a row, the second with a smaller input, in all storage
forms and on both lattices."""
import ctypes

import pytest
import torch

import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

BASE = dict(rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0, gamma_even=0.0)


def _views(reps, pool, storage, lattice):
    """Per-replica state views into a pool laid out as for an Ensemble."""
    params = [lb.make_params(storage=storage, lattice=lattice, **r) for r in reps]
    arr = (lb.LbParams * len(params))(*params)
    q = lb.LATTICE_QD[lattice][0]
    out = []
    for i, p in enumerate(params):
        off = lb.lib().lb_batch_offset(arr, len(params), i)
        n = lb.lib().lb_state_bytes(ctypes.byref(p))
        out.append(pool[off:off + n].view(lb.STORAGE_DTYPE[storage]).view(q, p.nz, p.ny, p.nx))
    return out


@pytest.mark.parametrize("storage,lattice", [("f32", "d3q19"), ("f16", "d3q19"), ("bf16", "d3q19"), ("f32", "d2q9"),
                                             ("bf16", "d2q9")])
def test_noalloc_matches_context_steps(storage, lattice):
    two_d = lattice == "d2q9"
    big = [dict(BASE, nx=24, ny=24, nz=1 if two_d else 24, seed=1),
           dict(BASE, nx=17, ny=9, nz=1 if two_d else 5, seed=2, kT=1e-3, gamma_shear=0.3),
           dict(BASE, nx=300, ny=12, nz=1 if two_d else 7, seed=3)]
    # call 1: three lattices from t0 = 0, 21 steps (a run of 16 launches and a tail)
    ens = lbf.Ensemble(big, storage=storage, init="thermal", lattice=lattice)
    pool = ens.pool.clone()
    ens.step(21)
    lb.step_noalloc(big, pool, 0, 21, storage=storage, lattice=lattice)
    torch.cuda.synchronize()
    for r, v in enumerate(_views(big, pool, storage, lattice)):
        assert torch.equal(v, ens.replica_state(r)), (storage, lattice, r)
    ens.close()
    # call 2: one smaller lattice from an odd t0 = 5, 10 steps
    small = dict(BASE, nx=8, ny=6, nz=1 if two_d else 5, seed=4)
    lat = lbf.Lattice(**small, storage=storage, init="thermal", lattice=lattice)
    lat.step(5)
    s0 = lat.state.clone()
    free0 = torch.cuda.mem_get_info()[0]
    lb.step_noalloc([small], s0, 5, 10, storage=storage, lattice=lattice)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    lat.step(10)
    assert torch.equal(s0, lat.state), (storage, lattice)
    say(f"noalloc {storage} {lattice}: device free memory {free0} -> {free1}")
    assert free1 == free0
    lat.close()


def test_noalloc_largest_batch_and_limit():
    """64 lattices (the maximum) in one call; 65 are refused."""
    reps = [dict(BASE, nx=4 + (i % 5), ny=3 + (i % 4), nz=2 + (i % 3), seed=100 + i) for i in range(64)]
    ens = lbf.Ensemble(reps, storage="f32", init="thermal")
    pool = ens.pool.clone()
    ens.step(7)
    lb.step_noalloc(reps, pool, 0, 7)
    torch.cuda.synchronize()
    for r, v in enumerate(_views(reps, pool, "f32", "d3q19")):
        assert torch.equal(v, ens.replica_state(r)), r
    ens.close()
    with pytest.raises(lb.LBError) as ei:
        lb.step_noalloc(reps + [reps[0]], pool, 0, 1)
    assert ei.value.code == lb.LB_EUNSUPPORTED and "64" in str(ei.value)
