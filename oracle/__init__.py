"""FP64 CPU oracle for the fluctuating lattice Boltzmann update (D3Q19, D2Q9).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this package.  It loads
``liblbora.so`` (plain C, built from ``lbora.c`` by ``oracle/build.py``) and
shares nothing with the GPU library.

Arrays follow the layout [q][z][y][x] (x fastest) of absolute populations
n_i in float64.  Parameters mirror the paper's: rho0, kT (mu = kT / c_s^2 =
3 kT in lattice units, Sec. VI), the bulk and shear rates gamma_b and gamma_s
and the kinetic-mode rates (Sec. IV).

Pinned by tests/test_oracle_*.py against the paper's Tables I and II and weights,
the equilibrium moment identities (Sec. II), exact conservation (Eq.
conservationlaws), stationary mode variances mu rho w_k (Eq. modeprob with
Eqs. xdef and evectors_orthonormal), the single-site AR(1) law and random
stress covariances (Sec. IV), and the viscosities of Eqs. shearviscosity and
bulkviscosity through the decay of shear and sound waves.
"""
import ctypes
import os

import numpy as np

from . import build as _build

Q = 19
D3Q19, D2Q9 = 0, 1
LATTICE_QD = {D3Q19: (19, 3), D2Q9: (9, 2)}
HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class OraParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("rho0", ctypes.c_double), ("kT", ctypes.c_double),
        ("gamma_bulk", ctypes.c_double), ("gamma_shear", ctypes.c_double),
        ("gamma_odd", ctypes.c_double), ("gamma_even", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("thermal_modes", ctypes.c_int32), ("lattice", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        pp = ctypes.POINTER(OraParams)
        L.ora_tables.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp, dp, dp]
        L.ora_tables.restype = ctypes.c_int32
        L.ora_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.ora_uniform_chunks.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_int32, u32p]
        L.ora_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_int32, dp]
        L.ora_equilibrium.argtypes = [ctypes.c_int32, ctypes.c_double, dp, dp]
        L.ora_equilibrium.restype = ctypes.c_int
        L.ora_collide_site.argtypes = [pp, dp, ctypes.c_uint32, ctypes.c_uint64]
        L.ora_collide_site.restype = ctypes.c_int
        L.ora_step.argtypes = [pp, dp, dp, ctypes.c_uint64]
        L.ora_step.restype = ctypes.c_int64
        L.ora_run.argtypes = [pp, dp, dp, ctypes.c_uint64, ctypes.c_int64]
        L.ora_run.restype = ctypes.c_int64
        L.ora_init.argtypes = [pp, ctypes.c_int32, dp, dp]
        L.ora_init.restype = ctypes.c_int
        L.ora_moments.argtypes = [pp, dp, dp]
        L.ora_moments.restype = ctypes.c_int
        L.ora_modes.argtypes = [pp, dp, dp]
        L.ora_modes.restype = ctypes.c_int
        L.ora_num_threads.restype = ctypes.c_int32
        L.ora_set_num_threads.argtypes = [ctypes.c_int32]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u32p(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


INIT_REST, INIT_THERMAL, INIT_FIELDS = 0, 1, 2
THERMAL_ALL, THERMAL_STRESS_ONLY = 0, 1


def params(nx, ny, nz, rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=0.5,
           gamma_odd=0.0, gamma_even=0.0, seed=0, thermal_modes=THERMAL_ALL, lattice=D3Q19):
    return OraParams(nx, ny, nz, rho0, kT, gamma_bulk, gamma_shear,
                     gamma_odd, gamma_even, seed, thermal_modes, lattice)


def tables(lattice=D3Q19):
    """(c[q,3] int, a[q], e[q,q] as [k,i], w[q]) built from Table II (D3Q19)
    or Table I (D2Q9)."""
    q, _ = LATTICE_QD[lattice]
    c = np.zeros((q, 3), np.int32)
    a = np.zeros(q)
    e = np.zeros((q, q))
    w = np.zeros(q)
    got = lib().ora_tables(lattice, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(a), _dp(e), _dp(w))
    assert got == q
    return c, a, e, w


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_u32p(c), _u32p(k), _u32p(out))
    return out


def uniform_chunks(seed, site, t, stream, n):
    out = np.zeros(n, np.uint32)
    lib().ora_uniform_chunks(seed, site, t, stream, n, _u32p(out))
    return out


def normals(seed, site, t, stream, n):
    out = np.zeros(n + 1)
    lib().ora_normals(seed, site, t, stream, n, _dp(out))
    return out[:n]


def equilibrium(rho, u, lattice=D3Q19):
    """n^eq(rho, u) of Eq. derived_equil_distrib; u has three components."""
    u = np.zeros(3) + np.asarray(u, dtype=np.float64)
    out = np.zeros(LATTICE_QD[lattice][0])
    if lib().ora_equilibrium(lattice, float(rho), _dp(u), _dp(out)) != 0:
        raise ValueError("oracle: unknown lattice")
    return out


def collide_site(p, n, site, t):
    """Collide one site's q populations (copy returned); raises on rho <= 0."""
    v = np.array(n, dtype=np.float64)
    rc = lib().ora_collide_site(ctypes.byref(p), _dp(v), site, t)
    if rc == -2:
        raise ValueError("oracle: unusable parameters")
    if rc != 0:
        raise ValueError("oracle: rho <= 0 at site")
    return v


def shape(p):
    return (LATTICE_QD[p.lattice][0], int(p.nz), int(p.ny), int(p.nx))


def dim(p):
    return LATTICE_QD[p.lattice][1]


def init(p, kind, fields=None):
    n = np.zeros(shape(p))
    f = None
    if fields is not None:
        f = np.ascontiguousarray(fields, dtype=np.float64)
        assert f.shape == (1 + dim(p), p.nz, p.ny, p.nx)
    rc = lib().ora_init(ctypes.byref(p), kind, _dp(f) if f is not None else None, _dp(n))
    if rc != 0:
        raise ValueError("oracle: bad init kind or missing fields")
    return n


def step(p, n, t):
    out = np.empty_like(n)
    bad = lib().ora_step(ctypes.byref(p), _dp(n), _dp(out), t)
    return out, bad


def run(p, n, t0, nsteps):
    """Advance a copy of n by nsteps steps from step count t0."""
    s = np.array(n, dtype=np.float64, order="C")
    tmp = np.empty_like(s)
    bad = lib().ora_run(ctypes.byref(p), _dp(s), _dp(tmp), t0, nsteps)
    if bad < 0:
        raise ValueError("oracle: unusable parameters")
    if bad:
        raise ValueError(f"oracle: {bad} site-collisions with rho <= 0")
    return s


def moments(p, n):
    out = np.zeros((1 + dim(p), p.nz, p.ny, p.nx))
    if lib().ora_moments(ctypes.byref(p), _dp(np.ascontiguousarray(n)), _dp(out)) != 0:
        raise ValueError("oracle: unusable parameters")
    return out


def modes(p, n):
    out = np.zeros(shape(p))
    if lib().ora_modes(ctypes.byref(p), _dp(np.ascontiguousarray(n)), _dp(out)) != 0:
        raise ValueError("oracle: unusable parameters")
    return out


def num_threads():
    return int(lib().ora_num_threads())


def set_num_threads(n):
    lib().ora_set_num_threads(int(n))
