"""Host-side pieces of the benchmark: the one-GPU guard, the kernel-source
hash that ties stored counter values to the code they were taken on, and
the equilibrium stress modes its variance check subtracts."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import oracle  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_kernel_hash_ignores_comments_and_blank_space(tmp_path, monkeypatch):
    src = tmp_path / "k.h"
    src.write_text("// header\nint f(int a) {  /* doubled */\n  return 2 * a;   // twice\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.h"])
    h0 = bench.kernel_hash()
    src.write_text("/* other words */\nint f(int a) {\n    return 2 * a;\n}\n// trailing\n")
    assert bench.kernel_hash() == h0
    src.write_text("int f(int a) {\n  return 3 * a;\n}\n")
    assert bench.kernel_hash() != h0


def test_stress_equilibrium_matches_the_oracle_projection():
    """The benchmark's m_k^eq (stress modes from rho and j) equals the
    projection of the oracle's equilibrium populations, on both lattices."""
    rng = np.random.default_rng(3)
    for lattice, name, q, d in ((oracle.D3Q19, "d3q19", 19, 3), (oracle.D2Q9, "d2q9", 9, 2)):
        c, a, e, w = oracle.tables(lattice)
        for _ in range(5):
            rho = 1.0 + 0.1 * rng.standard_normal()
            u = 0.05 * rng.standard_normal(3)
            if d == 2:
                u[2] = 0.0
            n = oracle.equilibrium(rho, u, lattice)
            m = e @ n
            j = m[1:1 + d]
            for k in range(q):
                want = bench.stress_eq(name, k, j, m[0])
                if want is not None:
                    assert abs(m[k] - want) < 1e-12, (name, k)
