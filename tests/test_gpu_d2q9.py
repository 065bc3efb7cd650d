"""The D2Q9 lattice (basis of Table I) on the GPU: parity with the FP64
oracle element by element (trajectories, ragged and degenerate boxes, both
AA parities, every launch schedule), replicas of an ensemble, the stationary
law and the exact shear-wave decay, and sampled parity at the 2^28-site
throughput size.  Tolerance as for D3Q19: max |n_gpu - n_oracle| / (a_i rho0)
<= 1e-5 for fp32 state."""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
import workloads
from tests import lbtheory as th
from tests.gpu_util import gpu_pops, oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu
TOL = 1e-5
TABS = None


def tabs():
    global TABS
    if TABS is None:
        TABS = oracle.tables(oracle.D2Q9)
    return TABS


def cfg2(nx, ny, **kw):
    c = dict(nx=nx, ny=ny, nz=1, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5, gamma_odd=0.0,
             gamma_even=0.0, seed=7, lattice="d2q9")
    c.update(kw)
    return c


def run_pair(cfg, init, steps_list, fields=None, t0=0, storage="f32"):
    lat = lbf.Lattice(**cfg, storage=storage, init=init, t0=t0,
                      fields=None if fields is None else torch.from_numpy(fields))
    p = oracle_params(cfg)
    kind = {"rest": oracle.INIT_REST, "thermal": oracle.INIT_THERMAL, "fields": oracle.INIT_FIELDS}[init]
    n = oracle.init(p, kind, None if fields is None else fields.astype(np.float64))
    t, out = 0, []
    for target in steps_list:
        lat.step(target - t)
        n = oracle.run(p, n, t0 + t, target - t)
        t = target
        assert lat.t == t0 + t
        out.append((t, scaled_err(gpu_pops(lat), n, cfg["rho0"])))
    lat.close()
    return out


def test_trajectory_100_steps():
    cfg = dict(workloads.SMALL_2D)
    say("d2q9 parity: 64 x 48 rest, 100 steps")
    for t, err in run_pair(cfg, "rest", [1, 2, 3, 50, 99, 100]):
        say(f"  t={t}: err={err:.3e}")
        assert err < TOL, (t, err)


@pytest.mark.parametrize("dims", [(1, 1), (2, 2), (3, 5), (7, 1), (1, 6), (17, 13), (300, 7)])
def test_tiny_and_ragged_boxes(dims):
    cfg = cfg2(*dims, kT=1e-3, gamma_bulk=0.3, gamma_shear=0.7, gamma_odd=-0.2, gamma_even=0.4, seed=99)
    say(f"d2q9 parity: {dims} thermal")
    for t, err in run_pair(cfg, "thermal", [0, 1, 2, 5, 12]):
        assert err < TOL, (dims, t, err)


def test_fields_init_and_deterministic_wave():
    cfg = cfg2(6, 40, rho0=1.2, kT=0.0, gamma_shear=0.9, seed=0)
    f = workloads.random_fields(6, 40, 1, seed=3, rho0=1.2, dim=2)
    for t, err in run_pair(cfg, "fields", [0, 1, 2, 39, 80], fields=f):
        assert err < TOL, (t, err)


def test_stress_only_and_large_step_counter():
    cfg = cfg2(9, 8, thermal_modes="stress_only", seed=2 ** 33 + 5)
    for t, err in run_pair(cfg, "thermal", [1, 2, 20], t0=2 ** 32 + 3):
        assert err < TOL, (t, err)


def test_gathers_match_oracle():
    cfg = cfg2(9, 7, rho0=0.8, kT=5e-4, gamma_bulk=0.2, gamma_shear=0.6, gamma_odd=0.1, gamma_even=-0.1, seed=21)
    lat = lbf.Lattice(**cfg, init="thermal")
    p = oracle_params(cfg)
    n = oracle.init(p, oracle.INIT_THERMAL)
    for steps in (3, 4):
        lat.step(steps)
        n = oracle.run(p, n, lat.t - steps, steps)
        mom = lat.moments().double().cpu().numpy()
        assert mom.shape == (3, 1, 7, 9)
        np.testing.assert_allclose(mom, oracle.moments(p, n), atol=2e-6)
        np.testing.assert_allclose(lat.modes().double().cpu().numpy(), oracle.modes(p, n), atol=2e-6)
        nb, sums = lat.check()
        assert nb == 0 and sums[3] == 0.0
        np.testing.assert_allclose(sums[:3], oracle.moments(p, n).reshape(3, -1).sum(axis=1), rtol=1e-6, atol=1e-6)


def test_schedules_bit_identical():
    cfg = cfg2(300, 9, gamma_shear=0.8, seed=5)
    ref = lbf.Lattice(**cfg, init="thermal")
    for _ in range(37):
        ref.step(1)
    want = ref.state.clone()
    for sched in [dict(block=256, xcd_remap=1, graph_chunk=16), dict(block=64, xcd_remap=0, graph_chunk=4),
                  dict(block=512, xcd_remap=8, graph_chunk=2, tiling=1),
                  dict(block=128, xcd_remap=(0, 2), graph_chunk=10, tiling=(1, 0))]:
        lat = lbf.Lattice(**cfg, init="thermal")
        lat.set_schedule(**sched)
        lat.step(37)
        assert torch.equal(lat.state, want), sched
        lat.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_row_tiling_bit_identical(storage):
    cfg = cfg2(513, 3, gamma_odd=0.1, gamma_even=-0.2, seed=3)
    a = lbf.Lattice(**cfg, storage=storage, init="thermal")
    a.set_schedule(block=256, tiling=0)
    a.step(9)
    b = lbf.Lattice(**cfg, storage=storage, init="thermal")
    b.set_schedule(block=256, tiling=1)
    b.step(9)
    assert torch.equal(a.state, b.state)


def test_checkpoint_resume_and_ensemble_replicas():
    cfg = cfg2(20, 11, seed=11)
    full = lbf.Lattice(**cfg, init="thermal")
    full.step(30)
    part = lbf.Lattice(**cfg, init="thermal")
    part.step(13)
    snap, t = part.state.clone(), part.t
    part.close()
    resumed = lbf.Lattice(**cfg, init="keep", state=snap, t0=t)
    resumed.step(17)
    assert torch.equal(resumed.state, full.state)
    # replicas of one launch equal their standalone runs bit for bit
    reps = [dict(nx=20, ny=11, nz=1, kT=1e-4, seed=11, gamma_shear=0.5),
            dict(nx=64, ny=3, nz=1, kT=5e-4, seed=12, gamma_shear=0.8),
            dict(nx=1, ny=1, nz=1, kT=1e-3, seed=13, gamma_shear=0.1)]
    ens = lbf.Ensemble(reps, lattice="d2q9")
    ens.step(30)
    for r, rp in enumerate(reps):
        alone = lbf.Lattice(**rp, lattice="d2q9", init="thermal")
        alone.step(30)
        assert torch.equal(ens.replica_state(r), alone.state), r
        assert torch.equal(ens.view(r).populations(), alone.populations())
    ens.close()


def test_stationary_law_256():
    """Every mode's variance is mu rho0 w_k (conserved modes about their
    mean), and S(q) is flat at mu rho0, on a 256 x 256 lattice.  Snapshots
    are 50 steps apart; long waves decorrelate slowly, so each q-bin's
    standard error comes from the scatter of ten batch means."""
    c, a, e, w = tabs()
    L, kT = 256, 1e-4
    mu = 3 * kT
    cfg = cfg2(L, L, kT=kT, gamma_bulk=0.8, gamma_shear=-0.3, gamma_odd=0.4, gamma_even=-0.5, seed=4321)
    lat = lbf.Lattice(**cfg, init="thermal")
    var, sq = [], []
    for _ in range(200):
        lat.step(50)
        m = th.neq_modes_any(lat.modes().double().cpu().numpy(), 1.0, c, a, e)
        var.append(m.reshape(9, -1).var(axis=1))
        sq.append(np.abs(np.fft.fft2(m[0, 0])) ** 2 / L ** 2)
    lat.close()
    ratio = np.mean(var, axis=0) / (mu * w)
    say(f"d2q9 variance ratios {np.round(ratio, 4).tolist()}")
    assert np.abs(ratio - 1).max() < 0.01
    sq = np.array(sq) / mu
    kq = np.fft.fftfreq(L) * L
    kk = np.sqrt(kq[:, None] ** 2 + kq[None, :] ** 2)
    for lo, hi in [(0.5, 16), (16, 64), (64, 128), (128, 182)]:
        sel = (kk >= lo) & (kk < hi)
        per_snap = sq[:, sel].mean(axis=1)
        means = np.array([b.mean() for b in np.array_split(per_snap, 10)])
        se = means.std(ddof=1) / np.sqrt(10)
        say(f"  S(q)/mu rho0 for {lo} <= |k| < {hi}: {per_snap.mean():.4f} (se {se:.4f})")
        assert abs(per_snap.mean() - 1) < max(5 * se, 0.005) and abs(per_snap.mean() - 1) < 0.03, (lo, hi)


def test_shear_wave_decays_by_exact_eigenvalue():
    """kT = 0 shear wave u_x(y) on a 4 x 128 lattice: after the transient the
    amplitude shrinks per step by |lambda_T(q)| of the D2Q9 operator."""
    c, a, e, w = tabs()
    L, gs, U = 128, 0.9, 1e-3
    cfg = cfg2(4, L, kT=0.0, gamma_bulk=0.5, gamma_shear=gs)
    f = workloads.shear_wave_fields_2d(4, L, U)
    lat = lbf.Lattice(**cfg, init="fields", fields=torch.from_numpy(f))
    lat.step(200)
    y = np.arange(L)
    amps = []
    for _ in range(3):
        mom = lat.moments().double().cpu().numpy()
        amps.append((2.0 / (4 * L)) * (mom[1, 0] * np.sin(2 * np.pi * y / L)[:, None]).sum())
        lat.step(1)
    lam = abs(th.shear_eigenvalue(L, 1, th.mode_gammas(0.5, gs, 0, 0, q=9), c, a, e, w, axis=1))
    say(f"d2q9 shear decay {amps[1] / amps[0]:.8f} vs |lambda| {lam:.8f}")
    assert amps[1] / amps[0] == pytest.approx(lam, abs=1e-5)
    assert amps[2] / amps[1] == pytest.approx(lam, abs=1e-5)


def _sampled_step(lat, cfg, pts, tol):
    """One GPU step; the oracle collides the sampled sites' populations and
    Eq. LBE puts them at r + c_i, which must match the GPU's state."""
    c, a, e, w = tabs()
    nx, ny = cfg["nx"], cfg["ny"]
    t = lat.t
    pops = lat.populations()
    idx = torch.as_tensor(pts, device=pops.device)
    before = pops[:, 0, idx[:, 1], idx[:, 0]].double().cpu().numpy()
    del pops
    lat.step(1)
    pops = lat.populations()
    p = oracle_params(cfg)
    dest = []
    for k in range(len(pts)):
        x, y = (int(v) for v in pts[k])
        post = oracle.collide_site(p, before[:, k], x + nx * y, t)
        for i in range(9):
            dest.append((i, (y + c[i, 1]) % ny, (x + c[i, 0]) % nx, post[i], a[i]))
    d = np.array(dest)
    dev = pops.device
    got = pops[torch.as_tensor(d[:, 0].astype(np.int64), device=dev), 0,
               torch.as_tensor(d[:, 1].astype(np.int64), device=dev),
               torch.as_tensor(d[:, 2].astype(np.int64), device=dev)].double().cpu().numpy()
    del pops
    torch.cuda.empty_cache()
    worst = float((np.abs(got - d[:, 3]) / (d[:, 4] * cfg["rho0"])).max())
    say(f"  t={t} -> {t + 1}: {len(pts)} sites, max scaled err {worst:.3e}")
    assert worst < tol, worst


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("bf16", 2.0 ** -8)])
def test_full_size_sampled_parity(storage, tol):
    """16384 x 16384 (2^28 sites), default schedule, both parities, with
    samples on the faces where the periodic wrap happens."""
    cfg = dict(workloads.LARGE_2D)
    say(f"d2q9 16384^2 {storage}")
    lat = lbf.Lattice(**cfg, storage=storage, init="thermal")
    L = cfg["nx"]
    rng = np.random.default_rng(17)
    pts = np.vstack([rng.integers(0, L, size=(1500, 2)),
                     np.array([(0, 0), (L - 1, L - 1), (0, L - 1), (L - 1, 0), (0, 77), (L - 1, 5), (9, 0),
                               (3, L - 1)])])
    _sampled_step(lat, cfg, pts, tol)
    lat.step(17)
    lat.step(1)
    _sampled_step(lat, cfg, pts, tol)
    assert lat.check()[0] == 0
    lat.close()
