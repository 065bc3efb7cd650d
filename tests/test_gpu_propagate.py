"""Propagation only (lb_propagate): the streaming half of the update with the
identity collision moves every population n_i from r to r + c_i, periodic,
so the state after k such steps is the initial one with each population
field rolled by k c_i, bit for bit, on both lattices, in every storage form,
from either AA parity, for single lattices and batches."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb
from tests.gpu_util import LATTICES, gpu_pops, oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu


def velocities(lattice):
    c = np.asarray(oracle.tables(LATTICES[lattice])[0], dtype=np.int64)
    if c.shape[1] == 2:
        c = np.concatenate([c, np.zeros((len(c), 1), dtype=np.int64)], axis=1)
    return c


def rolled(pops, c, k):
    """n_i(r + k c_i) = n_i(r) on the periodic box; pops is (q, nz, ny, nx)."""
    out = torch.empty_like(pops)
    for i in range(pops.shape[0]):
        out[i] = torch.roll(pops[i], shifts=(int(k * c[i, 2]), int(k * c[i, 1]), int(k * c[i, 0])), dims=(0, 1, 2))
    return out


CASES = [("d3q19", (7, 5, 6)), ("d3q19", (16, 16, 16)), ("d3q19", (1, 1, 1)), ("d3q19", (33, 2, 3)),
         ("d2q9", (13, 11, 1)), ("d2q9", (64, 3, 1))]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("lattice,dims", CASES)
def test_stream_is_the_exact_shift(lattice, dims, storage):
    nx, ny, nz = dims
    c = velocities(lattice)
    for start_odd in (False, True):
        lat = lbf.Lattice(nx, ny, nz, storage=storage, kT=1e-3, gamma_shear=0.3, seed=17, lattice=lattice,
                          init="thermal")
        if start_odd:
            lat.step(1)
        t0 = lat.t
        p0 = lat.populations().clone()
        done = 0
        for k in (1, 2, 3):
            lat.propagate(k)
            done += k
            assert lat.t == t0 + done
            assert torch.equal(lat.populations(), rolled(p0, c, done)), (lattice, dims, storage, start_odd, done)
        lat.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_stream_period_returns_the_state(storage):
    """L propagation steps on an L-periodic cube bring every population back
    to where it started; with L even the parity, and so the stored layout,
    is the initial one as well, so the raw state returns bit for bit."""
    L = 12
    lat = lbf.Lattice(L, L, L, storage=storage, kT=1e-4, gamma_shear=0.5, seed=5, init="thermal")
    s0 = lat.state.clone()
    p0 = lat.populations().clone()
    lat.propagate(L)
    assert torch.equal(lat.state, s0)
    assert torch.equal(lat.populations(), p0)
    lat.close()


def test_stream_then_step_matches_oracle_shift():
    """A propagation step followed by an ordinary step: the ordinary step sees
    the shifted state and draws the noise of the advanced step count, as the
    oracle does from the rolled initial state at t = 1."""
    cfg = dict(nx=9, ny=8, nz=7, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0,
               gamma_even=0.0, seed=23)
    lat = lbf.Lattice(**cfg, init="thermal")
    p = oracle_params(cfg)
    n0 = oracle.init(p, oracle.INIT_THERMAL)
    c = velocities("d3q19")
    n1 = np.stack([np.roll(n0[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2)) for i in range(19)])
    lat.propagate(1)
    assert scaled_err(gpu_pops(lat), n1, 1.0) < 1e-6
    lat.step(2)
    want = oracle.run(p, n1, 1, 2)
    err = scaled_err(gpu_pops(lat), want, 1.0)
    say(f"stream + 2 steps vs oracle: {err:.2e}")
    assert err < 1e-5
    lat.close()


def test_batch_stream_moves_every_replica():
    reps = [dict(nx=16, ny=16, nz=16, kT=1e-4, gamma_shear=0.5, seed=1),
            dict(nx=5, ny=3, nz=7, kT=1e-3, gamma_shear=0.9, seed=2),
            dict(nx=1, ny=1, nz=1, kT=5e-4, gamma_shear=0.1, seed=3),
            dict(nx=32, ny=8, nz=9, kT=1e-5, gamma_shear=-0.5, seed=4)]
    c = velocities("d3q19")
    ens = lbf.Ensemble(reps, storage="f16", init="thermal")
    ens.step(3)
    p0 = [ens.view(r).populations().clone() for r in range(len(reps))]
    ens.propagate(5)
    assert ens.t == 8
    for r in range(len(reps)):
        assert torch.equal(ens.view(r).populations(), rolled(p0[r], c, 5)), r
    ens.close()


def test_stream_argument_errors():
    lat = lbf.Lattice(4, 4, 4, init="rest")
    with pytest.raises(lb.LBError) as ei:
        lat.propagate(-1)
    assert ei.value.code == lb.LB_EINVAL
    lat.propagate(0)
    assert lat.t == 0
    lat.close()
    ens = lbf.Ensemble([dict(nx=4, ny=4, nz=4), dict(nx=3, ny=3, nz=3)], init="rest")
    assert lb.lib().lb_propagate(ens.view(1)._ctx, 1) == lb.LB_EINVAL   # views cannot move; their batch can
    assert ens.t == 0
    ens.close()


def test_copy_rate_copies_and_reports_a_rate():
    """The copy calibration moves the bytes exactly and reports a positive
    rate below the HBM peak (read + write counted)."""
    n = (64 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    out = ctypes.c_double(0.0)
    rc = lb.lib().lb_copy_rate(lb._aligned(src), lb._aligned(dst), 4 * n, 3,
                               torch.cuda.current_stream().cuda_stream, ctypes.byref(out))
    assert rc == lb.LB_OK
    assert torch.equal(src, dst)
    assert 0.0 < out.value < 8000.0 * 1.05
    rate = lb.copy_rate(gib=1, reps=3)
    say(f"device copy, 1 GiB: {rate:.0f} GB/s")
    assert 1000.0 < rate < 8000.0 * 1.05


@pytest.mark.parametrize("lattice,dims", [("d3q19", (9, 7, 6)), ("d2q9", (17, 12, 1))])
def test_identity_collision_step_equals_propagation(lattice, dims):
    """With every rate gamma_k = 1 and kT = 0 the collision is the identity,
    so lb_step and lb_propagate agree up to the rounding of the mode
    transform round trip in fp32 (relative 1e-6 of a_i rho0)."""
    nx, ny, nz = dims
    cfg = dict(rho0=1.0, kT=0.0, gamma_bulk=1.0, gamma_shear=1.0, gamma_odd=1.0, gamma_even=1.0, seed=9,
               lattice=lattice)
    f = torch.zeros((3 if lattice == "d2q9" else 4, nz, ny, nx), dtype=torch.float32)
    g = torch.Generator().manual_seed(4)
    f[0] = 1.0 + 0.05 * torch.rand((nz, ny, nx), generator=g)
    f[1:] = 0.05 * (torch.rand(f[1:].shape, generator=g) - 0.5)
    a = lbf.Lattice(nx, ny, nz, init="fields", fields=f, **cfg)
    b = lbf.Lattice(nx, ny, nz, init="fields", fields=f, **cfg)
    a.step(5)
    b.propagate(5)
    q = a.q
    w = torch.as_tensor(oracle.tables(LATTICES[lattice])[1], dtype=torch.float32, device="cuda").view(q, 1, 1, 1)
    err = float(((a.populations() - b.populations()).abs() / w).max())
    say(f"{lattice}: step with identity collision vs propagation, 5 steps: {err:.2e}")
    assert err < 1e-6
    a.close()
    b.close()
