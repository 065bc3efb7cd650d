"""Planes of 4 GiB or more (here 1024^3 fp32: 2^30 sites, 19 planes of
exactly 4 GiB, 81.6 GB of state) leave the buffer-descriptor path, whose
range is a 32-bit byte count, and run the 64-bit-offset global-memory
kernels.  Parity on sampled sites against the oracle's single-site update,
both AA parities, with the default schedule (flat tiling; the row tiling is
refused for such planes)."""
import numpy as np
import pytest
import torch

import paper_0707_1581_amd as lbf
from paper_0707_1581_amd import lb
from tests.gpu_util import say
from tests.test_gpu_fullsize import check_one_step, sample_sites

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
    assert sched["tiling"] == [0, 0]
    with pytest.raises(lb.LBError) as ei:
        lat.set_schedule(block=256, tiling=1)
    assert ei.value.code == lb.LB_EUNSUPPORTED
    pts = sample_sites(L, 600, seed=9)
    check_one_step(lat, cfg, pts, 1e-5)      # even step
    lat.step(18)                             # one direct step, one 16-step graph replay, one more: t = 19
    check_one_step(lat, cfg, pts, 1e-5)      # odd step
    assert lat.check()[0] == 0
    lat.close()
