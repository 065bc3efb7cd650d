"""Parity at the full benchmark sizes, on sampled outputs the oracle computes
one by one: for sampled sites r the oracle collides the GPU's populations
n(r, t) (one site, the paper's update rule, noise keyed on (seed, site, t))
and Eq. LBE puts the result at r + c_i at step t + 1, which must equal the
GPU's state there.  Both AA parities are covered (t even and odd), with
the launch schedules the benchmark uses; samples include the faces and
edges where the periodic wrap happens."""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
import workloads
from tests.gpu_util import oracle_params, say

pytestmark = pytest.mark.gpu


def sample_sites(L, n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, L, size=(n, 3))
    edges = [(0, 0, 0), (L - 1, L - 1, L - 1), (0, L - 1, 0), (L - 1, 0, L - 1), (0, 5, 7), (L - 1, 9, 3),
             (4, 0, 2), (6, L - 1, 1), (3, 2, 0), (8, 1, L - 1)]
    return np.vstack([pts, np.array(edges)])


def check_one_step(lat, cfg, pts, tol):
    """Run one GPU step from the current t and compare the sampled sites."""
    L = cfg["nx"]
    c, a, e, w = oracle.tables()
    t = lat.t
    pops = lat.populations()
    idx = torch.as_tensor(pts, device=pops.device)
    before = pops[:, idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()  # (19, n)
    del pops
    lat.step(1)
    pops = lat.populations()
    p = oracle_params(cfg)
    worst = 0.0
    dest = []
    for k in range(len(pts)):
        x, y, z = (int(v) for v in pts[k])
        site = x + L * (y + L * z)
        post = oracle.collide_site(p, before[:, k], site, t)
        for i in range(19):
            dest.append((i, (z + c[i, 2]) % L, (y + c[i, 1]) % L, (x + c[i, 0]) % L, post[i], a[i]))
    d = np.array(dest)
    got = pops[torch.as_tensor(d[:, 0].astype(np.int64), device=pops.device),
               torch.as_tensor(d[:, 1].astype(np.int64), device=pops.device),
               torch.as_tensor(d[:, 2].astype(np.int64), device=pops.device),
               torch.as_tensor(d[:, 3].astype(np.int64), device=pops.device)].double().cpu().numpy()
    del pops
    torch.cuda.empty_cache()
    err = np.abs(got - d[:, 4]) / (d[:, 5] * cfg["rho0"])
    worst = float(err.max())
    say(f"  t={t} -> {t + 1}: {len(pts)} sites, max scaled err {worst:.3e}")
    assert worst < tol, worst


@pytest.mark.parametrize("remap,rows,resident", [(None, None, 0), (0, 0, 0), (1, 1, 0), (0, (1, 0), 1)])
def test_512_fp32_sampled_parity(remap, rows, resident):
    """None: the library's default schedule (the one the benchmark starts its
    tuning from); resident: the kernels of the resident cache policy."""
    cfg = dict(workloads.LARGE)
    say(f"512^3 fp32, xcd_remap={remap}, tiling={rows}, resident={resident}")
    lat = lbf.Lattice(**cfg, storage="f32", init="thermal")
    if remap is not None:
        lat.set_schedule(block=256, order=0, xcd_remap=remap, graph_chunk=16, tiling=rows, resident=resident)
    pts = sample_sites(512, 1500, seed=100 if remap is None else remap + 10 * resident)
    check_one_step(lat, cfg, pts, 1e-5)      # even step (t = 0)
    lat.step(17)                             # one direct step and one 16-step graph replay: t = 18
    lat.step(1)                              # t = 19
    check_one_step(lat, cfg, pts, 1e-5)      # odd step
    nb, _ = lat.check()
    assert nb == 0
    lat.close()


def test_768_fp16_sampled_parity():
    """fp16 storage: the oracle collides the stored (already rounded)
    populations exactly; the GPU's output differs by fp32 arithmetic plus
    one fp16 rounding of each stored d_i (relative 2^-11 of |d_i| <~ 1)."""
    cfg = dict(workloads.XLARGE)
    say("768^3 fp16, row tiling")
    lat = lbf.Lattice(**cfg, storage="f16", init="thermal")
    lat.set_schedule(block=256, order=0, xcd_remap=1, graph_chunk=16, tiling=1)
    pts = sample_sites(768, 800, seed=5)
    check_one_step(lat, cfg, pts, 2.0 ** -11)
    lat.step(2)
    check_one_step(lat, cfg, pts, 2.0 ** -11)
    lat.close()
