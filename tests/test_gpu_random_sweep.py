"""A seeded sweep over random configurations.

Each case draws a lattice (D3Q19 or D2Q9) and a box of 1 to 40 (D2Q9: 1 to
119) sites a side. It also draws rho0, rates in [-1, 1] for every mode class,
a temperature (kT = 0 runs start from random fields), all-mode or
stress-only noise, a 64-bit seed, a start time (0, odd, or just below the
step counter's 2^32 boundary), 1 to 9 steps, and a random launch schedule:
block, XCD remaps, tilings, cache policy, graph chunk and the fused
two-step pass.

fp32 cases are compared with the FP64 oracle to 1e-5 of a_i rho0. 16-bit
cases are compared, bit for bit, with the same configuration under the
default schedule."""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
from tests.gpu_util import gpu_pops, oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu

CASES = 36


def _case(k):
    rng = np.random.default_rng(7000 + k)
    lattice = "d2q9" if k % 3 == 2 else "d3q19"
    if lattice == "d3q19":
        nx, ny, nz = (int(v) for v in rng.integers(1, 41, size=3))
    else:
        nx, ny = (int(v) for v in rng.integers(1, 120, size=2))
        nz = 1
    kT = float(rng.choice([0.0, 1e-5, 1e-4, 1e-3]))
    cfg = dict(nx=nx, ny=ny, nz=nz, rho0=float(rng.uniform(0.5, 2.0)), kT=kT,
               gamma_bulk=float(rng.uniform(-1, 1)), gamma_shear=float(rng.uniform(-1, 1)),
               gamma_odd=float(rng.uniform(-1, 1)), gamma_even=float(rng.uniform(-1, 1)),
               seed=int(rng.integers(0, 2 ** 63)), lattice=lattice,
               thermal_modes=str(rng.choice(["all", "stress_only"])))
    storage = str(rng.choice(["f32", "f32", "f16", "bf16"]))
    t0 = int(rng.choice([0, 1, 7, 2 ** 32 - 3]))
    steps = int(rng.integers(1, 10))
    sched = dict(block=int(rng.choice([64, 128, 256, 512])), order=0,
                 xcd_remap=(int(rng.choice([0, 1, 2, 8])), int(rng.choice([0, 1, 2, 8]))),
                 graph_chunk=int(rng.choice([2, 4, 16])),
                 tiling=(int(rng.integers(0, 2)), int(rng.integers(0, 2))),
                 resident=int(rng.integers(0, 2)), group_mb=0, fused=int(rng.integers(0, 2)))
    fields = None
    if kT == 0.0:  # a deterministic start away from rest
        d = 2 if lattice == "d2q9" else 3
        f = np.empty((1 + d, nz, ny, nx), dtype=np.float32)
        f[0] = cfg["rho0"] * (1.0 + 0.01 * rng.standard_normal((nz, ny, nx)))
        f[1:] = 0.01 * rng.standard_normal((d, nz, ny, nx))
        fields = f
    return cfg, storage, t0, steps, sched, fields


@pytest.mark.parametrize("k", range(CASES))
def test_random_configuration(k):
    cfg, storage, t0, steps, sched, fields = _case(k)
    say(f"case {k}: {cfg['lattice']} {cfg['nx']}x{cfg['ny']}x{cfg['nz']} {storage} kT={cfg['kT']} "
        f"{cfg['thermal_modes']} t0={t0} steps={steps} sched={sched}")
    init = "thermal" if cfg["kT"] > 0 else "fields"
    fkw = {} if fields is None else {"fields": torch.from_numpy(fields)}
    lat = lbf.Lattice(**cfg, storage=storage, init=init, t0=t0, **fkw)
    lat.set_schedule(**sched)
    assert lat.schedule()["fused"] == sched["fused"]
    lat.step(steps)
    assert lat.t == t0 + steps
    if storage == "f32":
        p = oracle_params(cfg)
        kind = oracle.INIT_THERMAL if init == "thermal" else oracle.INIT_FIELDS
        n = oracle.init(p, kind, None if fields is None else fields.astype(np.float64))
        n = oracle.run(p, n, t0, steps)
        err = scaled_err(gpu_pops(lat), n, cfg["rho0"])
        say(f"  oracle: {err:.3e}")
        assert err < 1e-5, err
    else:
        ref = lbf.Lattice(**cfg, storage=storage, init=init, t0=t0, **fkw)
        ref.step(steps)
        assert torch.equal(lat.state, ref.state)
        ref.close()
    lat.close()
