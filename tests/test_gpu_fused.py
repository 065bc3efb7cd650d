"""The fused two-step schedule: each launch applies Eq. LBE twice (collision
with noise, push) to a whole D3Q19 or D2Q9 lattice, reading the state once and
writing it once into a second buffer, and a second launch brings the state
back.

Pinned three ways:
  - bit for bit against the single-step (AA) schedule on boxes that exercise
    every tile edge, the periodic wrap, tiles wider than the box, odd starts,
    graph replays and their tails, in all three storage forms;
  - against the FP64 oracle: the 16^3 trajectory of the parity workload to
    1e-5, and at 512^3 sampled sites against the oracle's own evolution of
    the neighbourhood of each site over one pair of passes;
  - propagation only: a pair of passes with the identity collision moves
    every stored value by 4 c_i, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb
import workloads
from tests.gpu_util import gpu_pops, oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu

BOXES = [(16, 16, 16), (70, 13, 9), (1, 1, 1), (2, 2, 2), (5, 3, 2), (64, 21, 40), (130, 17, 33), (3, 29, 4)]


def _cfg(dims, seed=4321):
    nx, ny, nz = dims
    return dict(nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
                gamma_even=0.2, seed=seed)


@pytest.mark.parametrize("dims", BOXES)
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_fused_equals_single_steps(dims, storage):
    cfg = _cfg(dims)
    a = lbf.Lattice(**cfg, storage=storage, init="thermal")
    b = lbf.Lattice(**cfg, storage=storage, init="thermal")
    a.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=0)
    b.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    assert b.schedule()["fused"] == 1
    for n in (1, 3, 4, 7, 16, 21, 37):  # an odd start, tails shorter than a pair, graph replays
        a.step(n)
        b.step(n)
        assert a.t == b.t
        assert torch.equal(a.state, b.state), (dims, storage, a.t)
    assert b.check()[0] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("lattice,dims", [("d3q19", (70, 13, 9)), ("d2q9", (1000, 130, 1))])
@pytest.mark.parametrize("variant", [dict(kT=0.0, gamma_bulk=-0.4, gamma_shear=0.9),
                                     dict(thermal_modes="stress_only", gamma_odd=0.0, gamma_even=0.0),
                                     dict(gamma_bulk=1.0, gamma_shear=-1.0, gamma_odd=1.0, gamma_even=-1.0),
                                     dict(seed=2 ** 40 + 3)])
def test_fused_collision_branches(lattice, dims, variant):
    """The other branches of the collision under the fused pass: no noise
    (kT = 0), the stress-only model, rates of +-1 in every class, a 64-bit
    seed; from a large step count, so the counter's high word is set."""
    nx, ny, nz = dims
    cfg = dict(nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
               gamma_even=0.2, seed=99, lattice=lattice)
    cfg.update(variant)
    t0 = 2 ** 32 - 6
    a = lbf.Lattice(**cfg, storage="f32", init="thermal" if cfg["kT"] > 0 else "rest", t0=t0)
    b = lbf.Lattice(**cfg, storage="f32", init="thermal" if cfg["kT"] > 0 else "rest", t0=t0)
    if cfg["kT"] == 0:  # a deterministic start away from rest: a few noisy steps of a twin
        w = lbf.Lattice(**dict(cfg, kT=1e-4), storage="f32", init="thermal", t0=t0)
        w.step(2)
        a.state.copy_(w.state)
        b.state.copy_(w.state)
        w.close()
    a.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=0)
    b.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    for n in (4, 9, 16):
        a.step(n)
        b.step(n)
        assert torch.equal(a.state, b.state), (lattice, variant, a.t)
    assert a.t > 2 ** 32
    a.close()
    b.close()


@pytest.mark.parametrize("chunk", [2, 4, 6, 8, 30])
def test_fused_graph_chunks(chunk):
    """Chunks that are not a multiple of four run their last two steps as AA
    steps inside the replay; the state is back in the caller's buffer after
    every call."""
    cfg = _cfg((70, 13, 9), seed=77)
    a = lbf.Lattice(**cfg, storage="f32", init="thermal")
    b = lbf.Lattice(**cfg, storage="f32", init="thermal")
    a.set_schedule(block=128, xcd_remap=1, graph_chunk=chunk, tiling=1, fused=0)
    b.set_schedule(block=128, xcd_remap=1, graph_chunk=chunk, tiling=1, fused=1)
    for n in (2 * chunk + 1, chunk, 3):
        a.step(n)
        b.step(n)
        assert torch.equal(a.state, b.state), (chunk, a.t)
    a.close()
    b.close()


def test_fused_trajectory_matches_oracle():
    """The parity workload (16^3, rest start, kT = 1e-4, 100 steps) under the
    fused schedule matches the FP64 oracle to 1e-5 (scaled by a_i rho0)."""
    cfg = dict(workloads.SMALL)
    lat = lbf.Lattice(**cfg, storage="f32", init="rest")
    lat.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    p = oracle_params(cfg)
    n = oracle.init(p, oracle.INIT_REST)
    t = 0
    for target in (4, 8, 99, 100):
        lat.step(target - t)
        n = oracle.run(p, n, t, target - t)
        t = target
        err = scaled_err(gpu_pops(lat), n, cfg["rho0"])
        say(f"fused 16^3 t={t}: max scaled err {err:.2e}")
        assert err < 1e-5, (t, err)
    lat.close()


def test_fused_propagation_is_exact_shift():
    cfg = _cfg((64, 21, 40), seed=5)
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    lat.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    c = oracle.tables()[0]
    before = lat.populations().clone()
    for n in (4, 5, 8):
        lat.propagate(n)
        after = lat.populations()
        k = lat.t
        for i in range(19):
            want = torch.roll(before[i], shifts=(k * int(c[i, 2]), k * int(c[i, 1]), k * int(c[i, 0])),
                              dims=(0, 1, 2))
            assert torch.equal(after[i], want), (n, i)
    lat.close()


def _patch_oracle(p, L, center, before, t0, nsteps):
    """Evolve the (2 nsteps + 1)^3 neighbourhood of `center` (populations
    `before`, (19, W, W, W), absolute) with the oracle's single-site update
    and push streaming for nsteps steps from t0; returns the populations of
    the center site afterwards (the only site whose whole past is inside)."""
    c = oracle.tables()[0]
    W = 2 * nsteps + 1
    cur = before
    for s in range(nsteps):
        new = np.zeros_like(cur)
        lo, hi = s, W - s
        for z in range(lo, hi):
            for y in range(lo, hi):
                for x in range(lo, hi):
                    gx = (center[0] - nsteps + x) % L
                    gy = (center[1] - nsteps + y) % L
                    gz = (center[2] - nsteps + z) % L
                    post = oracle.collide_site(p, cur[:, z, y, x], gx + L * (gy + L * gz), t0 + s)
                    for i in range(19):
                        zz, yy, xx = z + c[i, 2], y + c[i, 1], x + c[i, 0]
                        if 0 <= zz < W and 0 <= yy < W and 0 <= xx < W:
                            new[i, zz, yy, xx] = post[i]
        cur = new
    return cur[:, nsteps, nsteps, nsteps]


@pytest.mark.parametrize("box", ["LARGE", "XLARGE"])
def test_fused_sampled_parity_full_size(box):
    """The benchmark's fp32 boxes (512^3 and 768^3) under their default
    (fused) schedule: one pair of passes from t = 0, and one AA step plus one
    pair from an odd t, checked at sampled sites (faces, edges and tile seams
    included) against the oracle's evolution of each site's neighbourhood,
    and the whole state bit for bit against the AA schedule."""
    cfg = dict(getattr(workloads, box))
    L = cfg["nx"]
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    assert lat.schedule()["fused"] == 1, lat.schedule()
    rng = np.random.default_rng(21)
    pts = np.vstack([rng.integers(0, L, size=(24, 3)), [[0, 0, 0], [L - 1, L - 1, L - 1], [0, L - 1, 3],
                                                         [L - 1, 0, L - 1], [63, 10, 31], [64, 9, 32]]])
    p = oracle_params(cfg)
    # from t = 0: one pair of passes; from t = 19: one AA step, then a pair of passes
    for t_start, R in ((0, 4), (19, 5)):
        if lat.t < t_start:
            lat.step(t_start - lat.t)
        off = np.arange(-R, R + 1)
        pops = lat.populations()
        patches = []
        for x, y, z in pts:
            iz = torch.as_tensor((z + off) % L, device=pops.device)[:, None, None]
            iy = torch.as_tensor((y + off) % L, device=pops.device)[None, :, None]
            ix = torch.as_tensor((x + off) % L, device=pops.device)[None, None, :]
            patches.append(pops[:, iz, iy, ix].double().cpu().numpy())
        del pops
        torch.cuda.empty_cache()
        t0 = lat.t
        lat.step(R)
        pops = lat.populations()
        idx = torch.as_tensor(pts, device=pops.device)
        got = pops[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
        del pops
        torch.cuda.empty_cache()
        a = oracle.tables()[1]
        worst = 0.0
        for k, center in enumerate(pts):
            want = _patch_oracle(p, L, center, patches[k], t0, R)
            worst = max(worst, float((np.abs(got[:, k] - want) / (a * cfg["rho0"])).max()))
        say(f"{L}^3 fused, t={t0} -> {t0 + R}: {len(pts)} sites, max scaled err {worst:.2e}")
        assert worst < 1e-5, worst
    # the whole state against the single-step schedule from the same start
    ref = lbf.Lattice(**cfg, storage="f32", init="thermal")
    ref.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=(1, 0), fused=0)
    ref.step(lat.t)
    assert torch.equal(lat.state, ref.state)
    assert lat.check()[0] == 0
    lat.close()
    ref.close()
    del lat, ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("lattice,dims", [("d3q19", (176, 176, 176)), ("d3q19", (256, 256, 256)),
                                          ("d3q19", (130, 1000, 40)), ("d2q9", (2048, 2048, 1)), ("d2q9", (1000, 3000, 1))])
def test_fused_tail_aware_chunks(lattice, dims):
    """Lattices with few rounds of tiles, where the host shortens the chunks
    a tile walks (z-planes or rows; 176^3: 20, 256^3: 22, 2048^2: 13): the
    fused schedule equals AA steps bit for bit."""
    nx, ny, nz = dims
    cfg = dict(nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
               gamma_even=0.2, seed=77, lattice=lattice)
    a = lbf.Lattice(**cfg, storage="f32", init="thermal")
    assert a.schedule()["fused"] == 1, a.schedule()
    b = lbf.Lattice(**cfg, storage="f32", init="thermal")
    b.set_schedule(**dict(b.schedule(), fused=0))
    for n in (5, 16):
        a.step(n)
        b.step(n)
        assert torch.equal(a.state, b.state), (dims, a.t)
    assert a.check()[0] == 0
    a.close()
    b.close()
    del a, b
    torch.cuda.empty_cache()


def test_fused_schedule_rules():
    base = dict(rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0, gamma_even=0.0, seed=9)
    # default: fp32 D3Q19 beyond the cache fused; cache-sized and 16-bit state one step per launch
    for dims, st, want in [((192, 192, 192), "f32", 1), ((156, 156, 156), "f32", 1), ((152, 152, 152), "f32", 0),
                           ((128, 128, 128), "f32", 0), ((256, 256, 256), "f16", 0)]:
        lat = lbf.Lattice(nx=dims[0], ny=dims[1], nz=dims[2], **base, storage=st, init="rest")
        assert lat.schedule()["fused"] == want, (dims, st, lat.schedule())
        lat.close()
    # D2Q9 likewise (4096^2 fp32: 604 MB; 2048^2: 151 MB, resident)
    for dims, st, want in [((4096, 4096), "f32", 1), ((1024, 1024), "f32", 1), ((724, 724), "f32", 0),
                           ((4096, 4096), "bf16", 0)]:
        lat = lbf.Lattice(nx=dims[0], ny=dims[1], nz=1, **base, storage=st, init="rest", lattice="d2q9")
        assert lat.schedule()["fused"] == want, (dims, st, lat.schedule())
        lat.close()
    # ensembles have no fused pass
    ens = lbf.Ensemble([dict(base, nx=16, ny=16, nz=16, seed=s) for s in range(2)], init="rest")
    with pytest.raises(lb.LBError) as ei:
        ens.set_schedule(fused=1)
    assert ei.value.code == lb.LB_EUNSUPPORTED
    ens.close()
    lat = lbf.Lattice(nx=16, ny=16, nz=16, **base, init="rest")
    with pytest.raises(lb.LBError) as ei:
        lat.set_schedule(fused=2)
    assert ei.value.code == lb.LB_EINVAL
    lat.close()
    # switching the fused schedule off releases the second buffer
    torch.cuda.synchronize()
    lat = lbf.Lattice(nx=384, ny=384, nz=384, **base, storage="f32", init="rest")  # 4.3 GB of state
    assert lat.schedule()["fused"] == 1
    torch.cuda.synchronize()
    free_on = torch.cuda.mem_get_info()[0]
    lat.set_schedule(fused=0)
    torch.cuda.synchronize()
    free_off = torch.cuda.mem_get_info()[0]
    nbytes = 19 * 384 ** 3 * 4
    assert free_off - free_on > 0.9 * nbytes, (free_on, free_off)
    lat.set_schedule(fused=1)
    assert lat.schedule()["fused"] == 1
    lat.close()


def test_autotune_tries_the_fused_schedule():
    cfg = _cfg((96, 96, 96), seed=3)
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    ref = lbf.Lattice(**cfg, storage="f32", init="thermal")
    import json
    rep = json.loads(lat.autotune(steps=4))
    stage2 = [r for r in rep if r.get("stage") == 2]
    assert any(r["fused"] == 1 for r in stage2), stage2
    say(f"96^3 fp32 stage 2: {[(r['resident'], r['fused'], round(r['ms_per_step'], 4)) for r in stage2]}, "
        f"picked {lat.schedule()}")
    # tuning left the state and the step count alone, and any choice gives the same trajectory
    assert lat.t == 0 and torch.equal(lat.state, ref.state)
    lat.step(20)
    ref.step(20)
    assert torch.equal(lat.state, ref.state)
    lat.close()
    ref.close()


# ---------------------------------------------------------------- D2Q9
BOXES_2D = [(1, 1), (2, 2), (5, 3), (256, 32), (257, 33), (1000, 130), (64, 200), (1030, 7), (3, 131)]


def _cfg2(dims, seed=4321):
    nx, ny = dims
    return dict(nx=nx, ny=ny, nz=1, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
                gamma_even=0.2, seed=seed, lattice="d2q9")


@pytest.mark.parametrize("dims", BOXES_2D)
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_fused_2d_equals_single_steps(dims, storage):
    """Segments that clip at the box edge, segments wider than the box, rows
    chunks shorter than a chunk, boxes of one row or column."""
    cfg = _cfg2(dims)
    a = lbf.Lattice(**cfg, storage=storage, init="thermal")
    b = lbf.Lattice(**cfg, storage=storage, init="thermal")
    a.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=0)
    b.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    assert b.schedule()["fused"] == 1
    for n in (1, 3, 4, 7, 16, 21, 37):
        a.step(n)
        b.step(n)
        assert a.t == b.t
        assert torch.equal(a.state, b.state), (dims, storage, a.t)
    assert b.check()[0] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("chunk", [2, 6, 30])
def test_fused_2d_graph_chunks(chunk):
    cfg = _cfg2((1000, 130), seed=77)
    a = lbf.Lattice(**cfg, storage="f32", init="thermal")
    b = lbf.Lattice(**cfg, storage="f32", init="thermal")
    a.set_schedule(block=128, xcd_remap=1, graph_chunk=chunk, tiling=1, fused=0)
    b.set_schedule(block=128, xcd_remap=1, graph_chunk=chunk, tiling=1, fused=1)
    for n in (2 * chunk + 1, chunk, 3):
        a.step(n)
        b.step(n)
        assert torch.equal(a.state, b.state), (chunk, a.t)
    a.close()
    b.close()


def test_fused_2d_trajectory_matches_oracle():
    """The D2Q9 parity workload (64 x 48, rest start, kT = 1e-4, 100 steps)
    under the fused schedule matches the FP64 oracle to 1e-5."""
    cfg = dict(workloads.SMALL_2D)
    lat = lbf.Lattice(**cfg, storage="f32", init="rest")
    lat.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    p = oracle_params(cfg)
    n = oracle.init(p, oracle.INIT_REST)
    t = 0
    for target in (4, 8, 99, 100):
        lat.step(target - t)
        n = oracle.run(p, n, t, target - t)
        t = target
        err = scaled_err(gpu_pops(lat), n, cfg["rho0"])
        say(f"fused d2q9 64x48 t={t}: max scaled err {err:.2e}")
        assert err < 1e-5, (t, err)
    lat.close()


def test_fused_2d_propagation_is_exact_shift():
    cfg = _cfg2((1000, 130), seed=5)
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    lat.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=0, fused=1)
    c = oracle.tables(oracle.D2Q9)[0]
    before = lat.populations().clone()
    for n in (4, 5, 8):
        lat.propagate(n)
        after = lat.populations()
        k = lat.t
        for i in range(9):
            want = torch.roll(before[i], shifts=(k * int(c[i, 1]), k * int(c[i, 0])), dims=(1, 2))
            assert torch.equal(after[i], want), (n, i)
    lat.close()


def _patch_oracle_2d(p, nx, ny, center, before, t0, nsteps):
    """The 2D form of _patch_oracle: evolve the (2 nsteps + 1)^2
    neighbourhood of `center` (populations `before`, (9, W, W)) with the
    oracle's single-site update and push streaming; returns the center's
    populations afterwards."""
    c = oracle.tables(oracle.D2Q9)[0]
    W = 2 * nsteps + 1
    cur = before
    for s in range(nsteps):
        new = np.zeros_like(cur)
        lo, hi = s, W - s
        for y in range(lo, hi):
            for x in range(lo, hi):
                gx = (center[0] - nsteps + x) % nx
                gy = (center[1] - nsteps + y) % ny
                post = oracle.collide_site(p, cur[:, y, x], gx + nx * gy, t0 + s)
                for i in range(9):
                    yy, xx = y + c[i, 1], x + c[i, 0]
                    if 0 <= yy < W and 0 <= xx < W:
                        new[i, yy, xx] = post[i]
        cur = new
    return cur[:, nsteps, nsteps]


def test_16384_fused_2d_sampled_parity():
    """The D2Q9 throughput box under its default (fused) schedule: one pair
    of passes from t = 0 and one AA step plus a pair from an odd t, checked
    at sampled sites (faces, corners and segment and chunk seams included)
    against the oracle's evolution of each site's neighbourhood, and the
    whole state bit for bit against the AA schedule."""
    cfg = dict(workloads.LARGE_2D)
    L = cfg["nx"]
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    assert lat.schedule()["fused"] == 1, lat.schedule()
    rng = np.random.default_rng(23)
    pts = np.vstack([rng.integers(0, L, size=(40, 2)),
                     [[0, 0], [L - 1, L - 1], [0, L - 1], [L - 1, 0], [255, 31], [256, 32], [511, 63]]])
    p = oracle_params(cfg)
    for t_start, R in ((0, 4), (19, 5)):
        if lat.t < t_start:
            lat.step(t_start - lat.t)
        off = np.arange(-R, R + 1)
        pops = lat.populations()
        patches = []
        for x, y in pts:
            iy = torch.as_tensor((y + off) % L, device=pops.device)[:, None]
            ix = torch.as_tensor((x + off) % L, device=pops.device)[None, :]
            patches.append(pops[:, 0, iy, ix].double().cpu().numpy())
        del pops
        torch.cuda.empty_cache()
        t0 = lat.t
        lat.step(R)
        pops = lat.populations()
        idx = torch.as_tensor(pts, device=pops.device)
        got = pops[:, 0, idx[:, 1], idx[:, 0]].double().cpu().numpy()
        del pops
        torch.cuda.empty_cache()
        a = oracle.tables(oracle.D2Q9)[1]
        worst = 0.0
        for k, center in enumerate(pts):
            want = _patch_oracle_2d(p, L, L, center, patches[k], t0, R)
            worst = max(worst, float((np.abs(got[:, k] - want) / (a * cfg["rho0"])).max()))
        say(f"16384^2 d2q9 fused, t={t0} -> {t0 + R}: {len(pts)} sites, max scaled err {worst:.2e}")
        assert worst < 1e-5, worst
    ref = lbf.Lattice(**cfg, storage="f32", init="thermal")
    ref.set_schedule(block=256, xcd_remap=0, graph_chunk=16, tiling=(1, 0), fused=0)
    ref.step(lat.t)
    assert torch.equal(lat.state, ref.state)
    assert lat.check()[0] == 0
    lat.close()
    ref.close()
