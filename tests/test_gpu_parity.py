"""Parity of the HIP path with the FP64 oracle, element by element, on the
same seeded inputs.  Tolerance for fp32 state: max_i,r |n_gpu - n_oracle| /
(a_i rho0) <= 1e-5 (scaling by a_i rho0 avoids near-zero denominators)."""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
import workloads
from tests.gpu_util import gpu_pops, oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu
TOL = 1e-5


def run_pair(cfg, init, steps_list, fields=None, t0=0, storage="f32"):
    """Yield (t, err) comparing GPU and oracle at each step count."""
    lat = lbf.Lattice(**cfg, storage=storage, init=init, t0=t0,
                      fields=None if fields is None else torch.from_numpy(fields))
    p = oracle_params(cfg)
    kind = {"rest": oracle.INIT_REST, "thermal": oracle.INIT_THERMAL, "fields": oracle.INIT_FIELDS}[init]
    n = oracle.init(p, kind, None if fields is None else fields.astype(np.float64))
    t = 0
    out = []
    for target in steps_list:
        lat.step(target - t)
        n = oracle.run(p, n, t0 + t, target - t)
        t = target
        assert lat.t == t0 + t
        out.append((t, scaled_err(gpu_pops(lat), n, cfg["rho0"])))
    lat.close()
    return out


def test_small_box_trajectory_100_steps():
    """16^3 periodic box, rest start, kT = 1e-4, gamma_s = gamma_b = 0.5,
    kinetic rates 0, seed 1234, 100 steps; checked at both AA parities."""
    cfg = dict(workloads.SMALL)
    say(f"parity: 16^3 rest, 100 steps")
    for t, err in run_pair(cfg, "rest", [1, 2, 3, 50, 99, 100]):
        say(f"  t={t}: err={err:.3e}")
        assert err < TOL, (t, err)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 5), (4, 3, 2), (1, 1, 7), (5, 1, 1),
                                  (1, 6, 1), (7, 3, 1), (17, 13, 11)])
def test_tiny_and_ragged_boxes(dims):
    """Boxes where neighbours alias (L = 1, 2) or the site count is not a
    multiple of the workgroup; thermal start, both parities."""
    nx, ny, nz = dims
    cfg = dict(nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-3, gamma_bulk=0.3, gamma_shear=0.7,
               gamma_odd=-0.2, gamma_even=0.4, seed=99)
    say(f"parity: {dims} thermal")
    for t, err in run_pair(cfg, "thermal", [0, 1, 2, 5, 12]):
        say(f"  t={t}: err={err:.3e}")
        assert err < TOL, (dims, t, err)


def test_fields_init_and_deterministic_wave():
    cfg = dict(nx=6, ny=5, nz=32, rho0=1.2, kT=0.0, gamma_bulk=0.5, gamma_shear=0.9,
               gamma_odd=0.0, gamma_even=0.0, seed=0)
    f = workloads.random_fields(6, 5, 32, seed=3, rho0=1.2)
    say("parity: random fields, kT = 0")
    for t, err in run_pair(cfg, "fields", [0, 1, 2, 31, 64], fields=f):
        say(f"  t={t}: err={err:.3e}")
        assert err < TOL, (t, err)


def test_stress_only_thermalisation():
    cfg = dict(nx=8, ny=8, nz=8, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5,
               gamma_odd=0.0, gamma_even=0.0, seed=7, thermal_modes="stress_only")
    say("parity: stress-only noise")
    for t, err in run_pair(cfg, "thermal", [1, 2, 20]):
        assert err < TOL, (t, err)


def test_large_step_counter():
    """Step counts above 2^32 use the high counter word."""
    cfg = dict(nx=4, ny=4, nz=4, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5,
               gamma_odd=0.0, gamma_even=0.0, seed=2 ** 33 + 5)
    say("parity: t0 = 2^32 + 3")
    for t, err in run_pair(cfg, "rest", [1, 2, 7], t0=2 ** 32 + 3):
        assert err < TOL, (t, err)


def test_gathers_match_oracle():
    cfg = dict(nx=9, ny=7, nz=5, rho0=0.8, kT=5e-4, gamma_bulk=0.2, gamma_shear=0.6,
               gamma_odd=0.1, gamma_even=-0.1, seed=21)
    lat = lbf.Lattice(**cfg, init="thermal")
    p = oracle_params(cfg)
    n = oracle.init(p, oracle.INIT_THERMAL)
    for steps in (3, 4):
        lat.step(steps)
        n = oracle.run(p, n, lat.t - steps, steps)
        mom = lat.moments().double().cpu().numpy()
        np.testing.assert_allclose(mom, oracle.moments(p, n), atol=2e-6)
        mod = lat.modes().double().cpu().numpy()
        np.testing.assert_allclose(mod, oracle.modes(p, n), atol=2e-6)
        nb, sums = lat.check()
        assert nb == 0
        om = oracle.moments(p, n).reshape(4, -1).sum(axis=1)
        np.testing.assert_allclose(sums, om, rtol=1e-6, atol=1e-6)


def test_graph_direct_and_schedules_bit_identical():
    """Graph replay vs single-step launches vs other launch schedules give
    the same bits (every site's arithmetic is the same)."""
    cfg = dict(nx=20, ny=9, nz=7, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8,
               gamma_odd=0.0, gamma_even=0.0, seed=5)
    ref = lbf.Lattice(**cfg, init="thermal")
    for _ in range(37):
        ref.step(1)
    want = ref.state.clone()
    for sched in [dict(block=256, xcd_remap=1, graph_chunk=16), dict(block=64, xcd_remap=0, graph_chunk=4),
                  dict(block=512, xcd_remap=1, graph_chunk=2), dict(block=128, xcd_remap=0, graph_chunk=36),
                  dict(block=256, xcd_remap=1, graph_chunk=16, tiling=1),
                  dict(block=64, xcd_remap=0, graph_chunk=6, tiling=1),
                  dict(block=256, xcd_remap=(0, 1), graph_chunk=16, tiling=(1, 0)),
                  dict(block=64, xcd_remap=(2, 4), graph_chunk=16, tiling=(0, 1)),
                  dict(block=128, xcd_remap=(3, 2), graph_chunk=10, tiling=(1, 1)),
                  dict(block=256, xcd_remap=0, graph_chunk=16, tiling=(1, 0), resident=1),
                  dict(block=64, xcd_remap=(2, 4), graph_chunk=4, tiling=(0, 1), resident=1),
                  dict(block=128, xcd_remap=1, graph_chunk=6, tiling=1, resident=1, group_mb=1)]:
        lat = lbf.Lattice(**cfg, init="thermal")
        lat.set_schedule(**sched)
        lat.step(37)
        assert torch.equal(lat.state, want), sched
        lat.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 5), (17, 13, 11), (64, 3, 2), (512, 2, 3)])
def test_row_tiling_bit_identical(storage, dims):
    """The row tiling (workgroups within one x-row, uniform y/z offsets)
    gives the same bits as the flat tiling."""
    nx, ny, nz = dims
    cfg = dict(nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.7,
               gamma_odd=0.1, gamma_even=-0.2, seed=3)
    a = lbf.Lattice(**cfg, storage=storage, init="thermal")
    a.set_schedule(block=256, tiling=0)
    a.step(9)
    b = lbf.Lattice(**cfg, storage=storage, init="thermal")
    b.set_schedule(block=256, tiling=1)
    b.step(9)
    assert torch.equal(a.state, b.state)


def test_checkpoint_resume_bit_identical():
    cfg = dict(nx=10, ny=10, nz=10, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5,
               gamma_odd=0.0, gamma_even=0.0, seed=11)
    full = lbf.Lattice(**cfg, init="thermal")
    full.step(30)
    part = lbf.Lattice(**cfg, init="thermal")
    part.step(13)
    snap, t = part.state.clone(), part.t
    part.close()
    resumed = lbf.Lattice(**cfg, init="keep", state=snap, t0=t)
    resumed.step(17)
    assert torch.equal(resumed.state, full.state)


@pytest.mark.parametrize("gammas", [(1.0, 1.0, 1.0, 1.0), (-1.0, -1.0, -1.0, -1.0), (1.0, -1.0, 0.0, 1.0),
                                    (0.0, 0.0, 0.0, 0.0)])
def test_extreme_rates(gammas):
    """|gamma| = 1 makes every noise amplitude sqrt(1 - gamma^2) zero (gamma = 1:
    no relaxation, pure streaming of a thermal state; gamma = -1: reflection
    about equilibrium); gamma = 0 relaxes fully in one step."""
    gb, gs, go, ge = gammas
    cfg = dict(nx=7, ny=6, nz=5, rho0=1.0, kT=1e-3, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go,
               gamma_even=ge, seed=77)
    for t, err in run_pair(cfg, "thermal", [1, 2, 9]):
        assert err < TOL, (gammas, t, err)


def test_zero_steps_is_a_no_op():
    cfg = dict(nx=9, ny=4, nz=3, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5, gamma_odd=0.0,
               gamma_even=0.0, seed=5)
    lat = lbf.Lattice(**cfg, init="thermal")
    lat.step(3)
    before = lat.state.clone()
    lat.step(0)
    assert lat.t == 3
    assert torch.equal(lat.state, before)
