"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark: the box configurations, the initial velocity / density fields of
deterministic waves, and the replica list of the ensemble workload.

This module holds no arithmetic of the update itself: it only produces
parameters and initial fields that both the GPU library and the CPU oracle
take as inputs.
"""
import numpy as np

# Lattice units: b = h = 1, c_s^2 = 1/3, mu = 3 kT.
BASE = dict(rho0=1.0, gamma_bulk=0.5, gamma_odd=0.0, gamma_even=0.0)

# 16^3 trajectory case, rest start, 100 steps.
SMALL = dict(BASE, nx=16, ny=16, nz=16, kT=1e-4, gamma_shear=0.5, seed=1234)
SMALL_STEPS = 100

# 128^3 shear-wave / statistics case.
MID = dict(BASE, nx=128, ny=128, nz=128, kT=1e-4, gamma_shear=0.5, seed=1234)

# 512^3 throughput case: thermal (random seeded rest) start, 200 steps.
LARGE = dict(BASE, nx=512, ny=512, nz=512, kT=1e-4, gamma_shear=0.8, seed=1234)
LARGE_STEPS = 200

# 768^3 16-bit storage case.
XLARGE = dict(BASE, nx=768, ny=768, nz=768, kT=1e-4, gamma_shear=0.8, seed=1234)

# D2Q9 (Table I) cases: a small trajectory case and a throughput case of
# 2^28 sites (9.66 GB of fp32 state, about the size of the 512^3 D3Q19 one).
SMALL_2D = dict(BASE, nx=64, ny=48, nz=1, kT=1e-4, gamma_shear=0.5, seed=1234, lattice="d2q9")
LARGE_2D = dict(BASE, nx=16384, ny=16384, nz=1, kT=1e-4, gamma_shear=0.8, seed=1234, lattice="d2q9")


def shear_wave_fields_2d(nx, ny, amplitude, periods=1, rho0=1.0):
    """(3, 1, ny, nx) float32: rho = rho0, u_x(y) = U sin(2 pi n y / ny)."""
    f = np.zeros((3, 1, ny, nx), dtype=np.float32)
    f[0] = rho0
    y = np.arange(ny)
    f[1] = (amplitude * np.sin(2 * np.pi * periods * y / ny)).astype(np.float32)[None, :, None]
    return f


def shear_wave_fields(nx, ny, nz, amplitude, periods=1, rho0=1.0):
    """(4, nz, ny, nx) float32: rho = rho0, u_x(z) = U sin(2 pi n z / nz)."""
    f = np.zeros((4, nz, ny, nx), dtype=np.float32)
    f[0] = rho0
    z = np.arange(nz)
    f[1] = (amplitude * np.sin(2 * np.pi * periods * z / nz)).astype(np.float32)[:, None, None]
    return f


def density_wave_fields(nx, ny, nz, amplitude, periods=1, rho0=1.0):
    """(4, nz, ny, nx) float32: rho = rho0 (1 + A sin(2 pi n z / nz)), u = 0."""
    f = np.zeros((4, nz, ny, nx), dtype=np.float32)
    z = np.arange(nz)
    f[0] = (rho0 * (1 + amplitude * np.sin(2 * np.pi * periods * z / nz))).astype(np.float32)[:, None, None]
    return f


def random_fields(nx, ny, nz, seed, drho=0.05, du=0.03, rho0=1.0, dim=3):
    """(1 + dim, nz, ny, nx) float32 smooth-free random density and velocity."""
    rng = np.random.default_rng(seed)
    f = np.empty((1 + dim, nz, ny, nx), dtype=np.float32)
    f[0] = rho0 * (1 + rng.uniform(-drho, drho, (nz, ny, nx)))
    f[1:] = rng.uniform(-du, du, (dim, nz, ny, nx))
    return f


ENSEMBLE_SIZES = (32, 48, 64, 96)


def ensemble_replicas(n=96, meta_seed=20070711, sizes=ENSEMBLE_SIZES, kT_range=(1e-5, 1e-3),
                      gamma_shear_range=(0.0, 0.9)):
    """Replica list of the ensemble workload: cubic boxes drawn uniformly
    from `sizes`, kT and gamma_shear uniform in their ranges, gamma_bulk 0.5,
    kinetic rates 0, distinct seeds; all drawn from one recorded meta-seed."""
    rng = np.random.default_rng(meta_seed)
    L = rng.choice(np.asarray(sizes), size=n)
    kT = rng.uniform(*kT_range, size=n)
    gs = rng.uniform(*gamma_shear_range, size=n)
    seeds = rng.choice(2 ** 40, size=n, replace=False)
    return [dict(nx=int(l), ny=int(l), nz=int(l), rho0=1.0, kT=float(k), gamma_bulk=0.5,
                 gamma_shear=float(g), gamma_odd=0.0, gamma_even=0.0, seed=int(s))
            for l, k, g, s in zip(L, kT, gs, seeds)]
