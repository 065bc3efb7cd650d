"""Property-based checks on the CPU (hypothesis): the oracle's collision
conserves mass and momentum and keeps a uniform equilibrium fixed for any
rates, density and velocity (Sec. II, Sec. IV), on both lattices; and the C
ABI's argument validation accepts exactly the documented parameter space,
reporting the state size q * sites * sizeof(storage), without touching any
device memory."""
import ctypes

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from paper_0707_1581_amd import lb

rates = st.floats(-1.0, 1.0)
LAT = st.sampled_from([oracle.D3Q19, oracle.D2Q9])


@settings(max_examples=60, deadline=None)
@given(LAT, rates, rates, rates, rates, st.floats(0.2, 3.0), st.floats(0.0, 1e-2),
       st.integers(0, 2 ** 40), st.integers(0, 2 ** 31), st.integers(0, 2 ** 40))
def test_collision_conserves_mass_and_momentum(lat, gb, gs, go, ge, rho, kT, seed, site, t):
    c, a, e, w = oracle.tables(lat)
    rng = np.random.default_rng(seed % 1000)
    n = a * rho * (1 + rng.normal(0, 0.1, len(a)))
    p = oracle.params(1, 1, 1, rho0=1.0, kT=kT, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go,
                      gamma_even=ge, seed=seed, lattice=lat)
    out = oracle.collide_site(p, n, site, t)
    assert abs(out.sum() - n.sum()) <= 1e-13 * n.sum()
    np.testing.assert_allclose(out @ c, n @ c, atol=1e-14)


@settings(max_examples=60, deadline=None)
@given(LAT, rates, rates, rates, rates, st.floats(0.2, 3.0),
       st.lists(st.floats(-0.1, 0.1), min_size=3, max_size=3))
def test_uniform_equilibrium_is_fixed_at_zero_temperature(lat, gb, gs, go, ge, rho, u):
    c, a, e, w = oracle.tables(lat)
    if lat == oracle.D2Q9:
        u = [u[0], u[1], 0.0]
    neq = oracle.equilibrium(rho, u, lat)
    p = oracle.params(1, 1, 1, kT=0.0, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go, gamma_even=ge,
                      lattice=lat)
    np.testing.assert_allclose(oracle.collide_site(p, neq, 0, 0), neq, atol=1e-14)


@settings(max_examples=300, deadline=None)
@given(st.integers(-3, 5000), st.integers(-3, 5000), st.integers(-3, 5000), st.integers(-1, 3),
       st.one_of(st.floats(-1.0, 3.0), st.just(float("nan")), st.just(float("inf"))),
       st.one_of(st.floats(-1e-3, 1e-2), st.just(float("nan")), st.just(float("inf"))),
       st.lists(st.one_of(st.floats(-1.5, 1.5), st.just(float("nan"))), min_size=4, max_size=4),
       st.integers(-1, 2), st.integers(-1, 2))
def test_parameter_validation(nx, ny, nz, storage, rho0, kT, g, thermal_modes, lattice):
    L = lb.lib()
    p = lb.LbParams(nx, ny, nz, storage, rho0, kT, g[0], g[1], g[2], g[3], 7, thermal_modes, lattice)
    q = {0: 19, 1: 9}.get(lattice)
    sites = nx * ny * nz
    valid = (nx >= 1 and ny >= 1 and nz >= 1 and storage in (0, 1, 2) and rho0 > 0 and np.isfinite(rho0)
             and kT >= 0 and np.isfinite(kT) and all(-1.0 <= x <= 1.0 for x in g)
             and thermal_modes in (0, 1) and q is not None and not (lattice == 1 and nz != 1)
             and sites <= 2 ** 32 - 1024)
    nbytes = L.lb_state_bytes(ctypes.byref(p))
    if valid:
        assert nbytes == q * sites * (4 if storage == 0 else 2)
    else:
        assert nbytes == 0
        ctx = ctypes.c_void_p()
        # never dereferenced: validation fails before anything is enqueued
        rc = L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 0, None, 0, ctypes.byref(ctx))
        assert rc in (lb.LB_EINVAL, lb.LB_EUNSUPPORTED) and ctx.value is None
