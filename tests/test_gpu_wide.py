"""Planes of 4 GiB or more (here 1024^3 fp32: 2^30 sites, 19 planes of
exactly 4 GiB, 81.6 GB of state) leave the plane-wide buffer-descriptor
path, whose range is a 32-bit byte count: the AA steps run the 64-bit-offset
global-memory kernels, and the fused two-step passes (the default schedule
there) address each plane one z-plane at a time.  Parity on sampled sites
against the oracle: AA steps of both parities against its single-site
update (flat tiling; the row tiling is refused for such planes), a pair of
fused passes against its evolution of each site's neighbourhood, and the
fused schedule bit for bit against AA steps; propagation-only steps as
exact shifts."""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb
from tests.gpu_util import oracle_params, say
from tests.test_gpu_fullsize import check_one_step, sample_sites
from tests.test_gpu_fused import _patch_oracle, _patch_oracle_2d

pytestmark = pytest.mark.gpu


def test_1024_fp32_wide_planes_sampled_parity():
    free, total = torch.cuda.mem_get_info()
    if free < 200 * 2 ** 30:
        pytest.skip("needs about 170 GB of free device memory")
    L = 1024
    cfg = dict(nx=L, ny=L, nz=L, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0,
               gamma_even=0.0, seed=4242)
    say("1024^3 fp32 (4 GiB planes, 64-bit offsets)")
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    sched = lat.schedule()
    assert sched["tiling"] == [0, 0] and sched["fused"] == 1, sched
    with pytest.raises(lb.LBError) as ei:
        lat.set_schedule(block=256, tiling=1)
    assert ei.value.code == lb.LB_EUNSUPPORTED
    with pytest.raises(lb.LBError) as ei:
        lat.set_schedule(block=256, tiling=0, resident=1)
    assert ei.value.code == lb.LB_EUNSUPPORTED
    lat.set_schedule(block=256, xcd_remap=0, tiling=0, fused=0)  # AA steps only (the 64-bit-offset kernels)
    pts = sample_sites(L, 600, seed=9)
    check_one_step(lat, cfg, pts, 1e-5)      # even step
    lat.step(18)                             # one direct step, one 16-step graph replay, one more: t = 19
    check_one_step(lat, cfg, pts, 1e-5)      # odd step
    assert lat.check()[0] == 0
    # the modes gather of the wide kernels agrees with the projected populations
    import oracle
    c, a, e, w = oracle.tables()
    idx = torch.as_tensor(pts, device="cuda")
    pops = lat.populations()
    n = pops[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    del pops
    torch.cuda.empty_cache()
    modes = lat.modes()
    m = modes[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    del modes
    torch.cuda.empty_cache()
    want = e @ (n - a[:, None] * cfg["rho0"])
    assert np.abs(m - want).max() < 1e-5, np.abs(m - want).max()  # fp32 rounding of the absolute n_i
    # propagation only on the 64-bit-offset kernels, both parities: after k
    # steps n_i(r) is the old n_i(r - k c_i), bit for bit
    pops = lat.populations()
    want = {k: torch.stack([pops[i, (idx[:, 2] - k * int(c[i, 2])) % L, (idx[:, 1] - k * int(c[i, 1])) % L,
                                 (idx[:, 0] - k * int(c[i, 0])) % L] for i in range(19)]) for k in (1, 2)}
    del pops
    torch.cuda.empty_cache()
    for k in (1, 2):
        say(f"  propagate, t = {lat.t}")
        lat.propagate(1)
        pops = lat.populations()
        got = pops[:, idx[:, 2], idx[:, 1], idx[:, 0]]
        del pops
        torch.cuda.empty_cache()
        assert torch.equal(got, want[k]), k
    lat.close()


def test_1024_fp32_wide_planes_noiseless():
    """The kT = 0 branch of the 64-bit-offset D3Q19 AA kernels (the collision
    branches at run time on whether the lattice is thermal): from a state
    away from rest (two thermal steps of a noisy twin), one step of each
    parity at sampled sites against the oracle's deterministic single-site
    update."""
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 200 * 2 ** 30:
        pytest.skip("needs about 170 GB of free device memory")
    L = 1024
    cfg = dict(nx=L, ny=L, nz=L, rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
               gamma_even=0.2, seed=4245)
    say("1024^3 fp32 kT = 0 (64-bit-offset AA kernels)")
    w = lbf.Lattice(**dict(cfg, kT=1e-4), storage="f32", init="thermal")
    w.set_schedule(block=256, xcd_remap=0, tiling=0, fused=0)
    w.step(2)
    lat = lbf.Lattice(**cfg, storage="f32", init="rest")
    lat.set_schedule(block=256, xcd_remap=0, tiling=0, fused=0)
    lat.state.copy_(w.state)
    w.close()
    del w
    torch.cuda.empty_cache()
    pts = sample_sites(L, 300, seed=10)
    check_one_step(lat, cfg, pts, 1e-5)      # even step
    check_one_step(lat, cfg, pts, 1e-5)      # odd step
    assert lat.check()[0] == 0
    lat.close()
    del lat
    torch.cuda.empty_cache()


def _fingerprint(state, L):
    """Per-plane sums of the raw 32-bit patterns, and whole z-planes and
    y-rows at the wrap and at tile and chunk seams, copied to the host."""
    sums = [int(state[i].view(torch.int32).sum(dtype=torch.int64)) for i in range(state.shape[0])]
    zs = torch.as_tensor([0, 1, 31, 32, 33, L - 1], device=state.device)
    ys = torch.as_tensor([0, 9, 10, 11, L - 1], device=state.device)
    return sums, state[:, zs].cpu(), state[:, :, ys].cpu()


def test_1024_fp32_fused_wide_planes():
    """The fused passes on 4 GiB planes (1024^3 fp32, where they are the
    default schedule): one pair of passes from t = 0 at sampled sites (faces,
    the last site and tile and chunk seams included) against the oracle's
    evolution of each site's 9^3 neighbourhood, read straight from the even
    AA state; then the state at t = 24 against AA steps from the same start,
    bit for bit in per-plane checksums and in whole planes and rows at the
    seams."""
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 180 * 2 ** 30:
        pytest.skip("needs about 170 GB of free device memory")
    L = 1024
    cfg = dict(nx=L, ny=L, nz=L, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
               gamma_even=0.2, seed=4243)
    say("1024^3 fp32 fused passes (4 GiB planes, one z-plane per descriptor)")
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    assert lat.schedule()["fused"] == 1, lat.schedule()
    c, a, e, w = oracle.tables()
    rng = np.random.default_rng(31)
    pts = np.vstack([rng.integers(0, L, size=(16, 3)),
                     [[0, 0, 0], [L - 1, L - 1, L - 1], [63, 9, 31], [64, 10, 32], [L - 1, 1019, 0], [0, L - 1, 33]]])
    R = 4
    off = np.arange(-R, R + 1)
    patches = []
    for x, y, z in pts:  # t = 0, even: plane i at site r holds d_i(r)
        iz = torch.as_tensor((z + off) % L, device="cuda")[:, None, None]
        iy = torch.as_tensor((y + off) % L, device="cuda")[None, :, None]
        ix = torch.as_tensor((x + off) % L, device="cuda")[None, None, :]
        d = lat.state[:, iz, iy, ix].double().cpu().numpy()
        patches.append(a[:, None, None, None] * cfg["rho0"] * (1.0 + d))
    lat.step(R)  # one pair of fused passes
    idx = torch.as_tensor(pts, device="cuda")
    got = lat.state[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
    got = a[:, None] * cfg["rho0"] * (1.0 + got)
    p = oracle_params(cfg)
    worst = 0.0
    for k, center in enumerate(pts):
        want = _patch_oracle(p, L, center, patches[k], 0, R)
        worst = max(worst, float((np.abs(got[:, k] - want) / (a * cfg["rho0"])).max()))
    say(f"  t=0 -> {R}: {len(pts)} sites, max scaled err {worst:.2e}")
    assert worst < 1e-5, worst
    lat.step(24 - lat.t)
    assert lat.check()[0] == 0
    fp = _fingerprint(lat.state, L)
    # propagation only under the fused schedule (one pair of identity-collision
    # passes from even t): every population moves by 4 c_i, read from the raw
    # even-layout state at sampled sites
    spts = torch.as_tensor(np.vstack([pts, rng.integers(0, L, size=(400, 3))]), device="cuda")
    before = {i: lat.state[i].clone() for i in (0, 1, 6, 7, 18)}
    lat.propagate(4)
    for i, plane in before.items():
        src = [(spts[:, k] - 4 * int(c[i, k])) % L for k in range(3)]
        assert torch.equal(lat.state[i, spts[:, 2], spts[:, 1], spts[:, 0]], plane[src[2], src[1], src[0]]), i
    del before
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ref = lbf.Lattice(**cfg, storage="f32", init="thermal")
    ref.set_schedule(block=256, xcd_remap=0, tiling=0, fused=0)
    ref.step(24)
    fr = _fingerprint(ref.state, L)
    ref.close()
    del ref
    torch.cuda.empty_cache()
    assert fp[0] == fr[0]
    assert torch.equal(fp[1], fr[1]) and torch.equal(fp[2], fr[2])


def test_32768_d2q9_fp32_fused_wide_planes():
    """The D2Q9 fused passes on 4 GiB planes (32768^2 fp32, one row per
    descriptor): one pair of passes from t = 0 at sampled sites against the
    oracle's evolution of each site's 9^2 neighbourhood, read from the even
    AA state; then the state at t = 24 bit for bit against AA steps."""
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 100 * 2 ** 30:
        pytest.skip("needs about 80 GB of free device memory")
    n = 32768
    cfg = dict(nx=n, ny=n, nz=1, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=-0.3,
               gamma_even=0.2, seed=4244, lattice="d2q9")
    say("D2Q9 32768^2 fp32 fused passes (4 GiB planes, one row per descriptor)")
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    assert lat.schedule()["fused"] == 1, lat.schedule()
    a = oracle.tables(oracle.D2Q9)[1]
    rng = np.random.default_rng(32)
    pts = np.vstack([rng.integers(0, n, size=(20, 2)),
                     [[0, 0], [n - 1, n - 1], [255, 31], [256, 32], [n - 1, 0], [0, n - 1]]])
    R = 4
    off = np.arange(-R, R + 1)
    patches = []
    for x, y in pts:
        iy = torch.as_tensor((y + off) % n, device="cuda")[:, None]
        ix = torch.as_tensor((x + off) % n, device="cuda")[None, :]
        d = lat.state[:, 0, iy, ix].double().cpu().numpy()
        patches.append(a[:, None, None] * cfg["rho0"] * (1.0 + d))
    lat.step(R)
    idx = torch.as_tensor(pts, device="cuda")
    got = lat.state[:, 0, idx[:, 1], idx[:, 0]].double().cpu().numpy()
    got = a[:, None] * cfg["rho0"] * (1.0 + got)
    p = oracle_params(cfg)
    worst = 0.0
    for k, center in enumerate(pts):
        want = _patch_oracle_2d(p, n, n, center, patches[k], 0, R)
        worst = max(worst, float((np.abs(got[:, k] - want) / (a * cfg["rho0"])).max()))
    say(f"  t=0 -> {R}: {len(pts)} sites, max scaled err {worst:.2e}")
    assert worst < 1e-5, worst
    lat.step(24 - lat.t)
    assert lat.check()[0] == 0
    sums = [int(lat.state[i].view(torch.int32).sum(dtype=torch.int64)) for i in range(9)]
    rows = lat.state[:, 0, torch.as_tensor([0, 31, 32, 33, n - 1], device="cuda")].cpu()
    cols = lat.state[:, 0, :, torch.as_tensor([0, 255, 256, n - 1], device="cuda")].cpu()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ref = lbf.Lattice(**cfg, storage="f32", init="thermal")
    ref.set_schedule(block=256, xcd_remap=0, tiling=0, fused=0)
    ref.step(24)
    assert sums == [int(ref.state[i].view(torch.int32).sum(dtype=torch.int64)) for i in range(9)]
    assert torch.equal(rows, ref.state[:, 0, torch.as_tensor([0, 31, 32, 33, n - 1], device="cuda")].cpu())
    assert torch.equal(cols, ref.state[:, 0, :, torch.as_tensor([0, 255, 256, n - 1], device="cuda")].cpu())
    ref.close()
    del ref
    torch.cuda.empty_cache()


def test_largest_site_count_d2q9_f16():
    """The largest lattice the 32-bit site index allows: D2Q9 65536 x 65535
    (4,294,901,760 sites, just below 2^32; fp16 planes of 8.6 GB, so the
    64-bit-offset kernels run).  A kT = 0 shear wave u_x(y) is independent
    of x, so sampled sites up to the last site index must follow the FP64
    1 x 65535 reduction (up to fp16 storage rounding) at both parities."""
    free, total = torch.cuda.mem_get_info()
    if free < 200 * 2 ** 30:
        pytest.skip("needs about 180 GB of free device memory")
    import oracle
    import workloads
    nx, ny, U, periods = 65536, 65535, 1e-2, 5
    cfg = dict(nx=nx, ny=ny, nz=1, rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0,
               gamma_even=0.0, seed=0, lattice="d2q9")
    say("D2Q9 65536 x 65535 fp16 (site index up to 2^32 - 65537)")
    f = torch.zeros((3, 1, ny, nx), dtype=torch.float32, device="cuda")
    f[0] = 1.0
    y = torch.arange(ny, device="cuda", dtype=torch.float64)
    f[1, 0] = (U * torch.sin(2 * np.pi * periods * y / ny)).float()[:, None]
    lat = lbf.Lattice(**cfg, storage="f16", init="fields", fields=f)
    torch.cuda.synchronize()
    del f
    lat._fields = None
    torch.cuda.empty_cache()
    p = oracle.params(1, ny, 1, rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=0.8, lattice=oracle.D2Q9)
    n = oracle.init(p, oracle.INIT_FIELDS,
                    workloads.shear_wave_fields_2d(1, ny, U, periods).astype(np.float64))
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.integers(0, nx, 400), [0, nx - 1, nx - 1, 0, nx - 1]])
    ys = np.concatenate([rng.integers(0, ny, 400), [0, ny - 1, 0, ny - 1, ny - 2]])
    t = 0
    for target in (1, 2, 3):
        lat.step(target - t)
        n = oracle.run(p, n, t, target - t)
        t = target
        mom = lat.moments()
        got = mom[1, 0, torch.as_tensor(ys, device="cuda"), torch.as_tensor(xs, device="cuda")].double().cpu().numpy()
        del mom
        torch.cuda.empty_cache()
        want = oracle.moments(p, n)[1, 0, ys, 0]
        err = float(np.abs(got - want).max())
        say(f"  t={t}: max |jx - jx_oracle| = {err:.3e} (U = {U})")
        assert err < 1e-2 * U, (t, err)
    nb, sums = lat.check()
    assert nb == 0
    lat.close()


def _raw_pops(state, parity, pts, L, c, opp):
    """Populations d_i (stored scaled deviations, as fp64) of the sampled
    sites read straight from the AA state: at even t population i of site r
    is plane i at r; at odd t it is plane opp(i) at r - c_i."""
    dev = state.device
    x, y, z = (torch.as_tensor(pts[:, k], device=dev) for k in range(3))
    out = []
    for i in range(len(c)):
        if parity == 0:
            out.append(state[i, z, y, x])
        else:
            out.append(state[int(opp[i]), (z - int(c[i, 2])) % L, (y - int(c[i, 1])) % L, (x - int(c[i, 0])) % L])
    return torch.stack(out).double().cpu().numpy()


def test_raw_aa_reader_matches_gathers():
    """The raw-state reader used below agrees with the library's
    parity-resolved populations gather on a small ragged box, at both AA
    parities (t even and odd)."""
    import oracle
    L = 7
    cfg = dict(nx=L, ny=L, nz=L, rho0=1.2, kT=1e-3, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0,
               gamma_even=0.0, seed=5)
    lat = lbf.Lattice(**cfg, storage="bf16", init="thermal")
    c, a, e, w = oracle.tables()
    opp = np.array([0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)])
    pts = np.array([(x, y, z) for z in range(L) for y in range(L) for x in range(L)])
    for t in range(3):
        assert lat.t == t
        d = _raw_pops(lat.state, t & 1, pts, L, c, opp)
        pops = lat.populations()
        want = pops[:, pts[:, 2], pts[:, 1], pts[:, 0]].double().cpu().numpy()
        got = a[:, None] * cfg["rho0"] * (1.0 + d)
        assert np.abs(got - want).max() < 1e-6, t
        lat.step(1)
    lat.close()


def test_largest_site_count_d3q19_bf16():
    """The largest D3Q19 lattice the 32-bit site index allows: 1625^3 =
    4,291,015,625 sites (2^32 - 1024 is the limit), bf16 planes of 8.6 GB
    (64-bit-offset kernels), 163 GB of state.  No gather fits beside it, so
    the sampled sites are read from the raw AA state: one step from t = 0
    and one from t = 1, each against the oracle's single-site update of the
    stored populations (noise keyed on the site index, up to the last one)
    within bf16 storage rounding (2^-9 of |d_i| <~ 1, plus fp32)."""
    torch.cuda.empty_cache()  # blocks cached by earlier tests count as used
    free, total = torch.cuda.mem_get_info()
    if free < 180 * 2 ** 30:
        pytest.skip("needs about 170 GB of free device memory")
    import oracle
    from tests.gpu_util import oracle_params
    L = 1625
    cfg = dict(nx=L, ny=L, nz=L, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0,
               gamma_even=0.0, seed=777)
    say("1625^3 bf16 (site index up to 2^32 - 3,951,672; 8.6 GB planes, 64-bit offsets)")
    lat = lbf.Lattice(**cfg, storage="bf16", init="thermal")
    assert lat.schedule()["tiling"] == [0, 0]
    c, a, e, w = oracle.tables()
    opp = np.array([0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)])
    assert all((c[opp[i]] == -c[i]).all() for i in range(19))
    pts = sample_sites(L, 500, seed=17)
    p = oracle_params(cfg)
    for t in (0, 1):
        assert lat.t == t
        before = _raw_pops(lat.state, t & 1, pts, L, c, opp)
        lat.step(1)
        # population i of site r goes to r + c_i
        dest = (pts[None, :, :] + c[:, None, :].astype(np.int64)) % L   # (19, n, 3)
        after = np.empty_like(before)
        for i in range(19):
            after[i] = _raw_pops(lat.state, (t + 1) & 1, dest[i], L, c, opp)[i]
        worst = 0.0
        for k in range(len(pts)):
            x, y, z = (int(v) for v in pts[k])
            site = x + L * (y + L * z)
            n = a * cfg["rho0"] * (1.0 + before[:, k])
            post = oracle.collide_site(p, n, site, t)
            worst = max(worst, float(np.abs(after[:, k] - (post / (a * cfg["rho0"]) - 1.0)).max()))
        say(f"  t={t} -> {t + 1}: {len(pts)} sites, max |d_gpu - d_oracle| = {worst:.3e}")
        assert worst < 2.0 ** -8, worst
    nb, _ = lat.check()
    assert nb == 0
    lat.close()
    del lat
    torch.cuda.empty_cache()
