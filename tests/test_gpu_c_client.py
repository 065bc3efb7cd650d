"""The C ABI driven from C alone: tests/c_client/lb_client.c (plain C99, the
HIP runtime for device memory and the stream, no Python, no torch) runs a
thermal lattice through lb_init, lb_get_schedule / lb_set_schedule, lb_step,
lb_check and lb_populations and writes the populations to a file.  Its
output must equal, bit for bit, what the Python binding computes for the same
configuration, and in fp32 match the FP64 oracle's trajectory to 1e-5 of
a_i rho0 (the parity bound of the step kernels)."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_0707_1581_amd as lbf
from tests.gpu_util import oracle_params, say, scaled_err

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "lb_client")
# what lb_client.c sets
PARAMS = dict(rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0, gamma_even=0.0, seed=1234)
CASES = [("d3q19", (12, 10, 9), "f32", 0, 21), ("d3q19", (12, 10, 9), "f32", 1, 21),
         ("d2q9", (13, 11, 1), "f32", 1, 21), ("d2q9", (70, 9, 1), "f32", 0, 8),
         ("d3q19", (20, 7, 5), "bf16", 1, 13), ("d3q19", (20, 7, 5), "f16", 0, 13)]


@pytest.mark.parametrize("lattice,dims,storage,fused,steps", CASES)
def test_c_client_matches_binding_and_oracle(lattice, dims, storage, fused, steps, tmp_path):
    if not os.path.exists(CLIENT):
        pytest.fail(f"{CLIENT} is not built (run __graft_entry__.build())")
    nx, ny, nz = dims
    out = tmp_path / "pops.bin"
    say(f"lb_client {lattice} {dims} {storage} fused={fused} steps={steps}")
    proc = subprocess.run([CLIENT, lattice, str(nx), str(ny), str(nz), storage, str(steps), str(fused), str(out)],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stderr
    say(proc.stdout.strip())
    m = re.search(r"t=(\d+) bad=(-?\d+)", proc.stdout)
    assert m and int(m.group(1)) == steps and int(m.group(2)) == 0, proc.stdout
    q = 19 if lattice == "d3q19" else 9
    got = np.fromfile(out, dtype=np.float32)
    assert got.size == q * nz * ny * nx
    got = got.reshape(q, nz, ny, nx)

    lat = lbf.Lattice(nx, ny, nz, storage=storage, init="thermal", lattice=lattice, **PARAMS)
    if fused:
        lat.set_schedule(**dict(lat.schedule(), fused=1))
    assert lat.schedule()["fused"] == fused
    lat.step(steps)
    want = lat.populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, want), np.abs(got - want).max()

    if storage == "f32":
        p = oracle_params(dict(nx=nx, ny=ny, nz=nz, lattice=lattice, **PARAMS))
        ref = oracle.run(p, oracle.init(p, oracle.INIT_THERMAL), 0, steps)
        err = scaled_err(got, ref, PARAMS["rho0"])
        say(f"  oracle: max |n - n_oracle| / (a_i rho0) = {err:.3g}")
        assert err < 1e-5
