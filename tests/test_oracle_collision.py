"""Pins of the oracle's collision and streaming against what the paper and
the mathematics fix: the equilibrium's moments (Sec. II, Eq.
equilibriumstress with the Euler stress), exact conservation (Eq.
conservationlaws), the textbook single-relaxation-time special case, pure
streaming (Eq. LBE with the identity collision reduces to a periodic shift),
the single-site AR(1) law of Eqs. updaterule / FDT / langevin, and the random
stress covariances of the D3Q19 worked example (Sec. IV)."""
import itertools

import numpy as np
import pytest

import oracle
from tests import lbtheory as th

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def test_equilibrium_moments(tabs):
    c, a, e, w = tabs
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.5, 2.0)
        u = rng.normal(0, 0.05, 3)
        neq = oracle.equilibrium(rho, u)
        assert neq.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(neq @ c, rho * u, atol=1e-15)
        Pi = np.einsum("i,ia,ib->ab", neq, c, c)
        np.testing.assert_allclose(Pi, rho * CS2 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_conservation_through_collision(tabs):
    c, a, e, w = tabs
    rng = np.random.default_rng(2)
    p = oracle.params(1, 1, 1, rho0=1.0, kT=1e-3, gamma_bulk=-0.3, gamma_shear=0.7,
                      gamma_odd=0.2, gamma_even=-0.4, seed=11)
    for s in range(200):
        n = a * (1 + rng.normal(0, 0.2, 19))
        out = oracle.collide_site(p, n, s, s * 7)
        assert out.sum() == pytest.approx(n.sum(), rel=1e-14)
        np.testing.assert_allclose(out @ c, n @ c, atol=1e-15)
        assert not np.allclose(out, n)


def test_srt_special_case(tabs):
    """kT = 0 and the same gamma for every non-conserved mode is the
    single-relaxation-time rule n* = n^eq + gamma (n - n^eq)."""
    c, a, e, w = tabs
    rng = np.random.default_rng(3)
    for g in (0.0, 0.5, -0.8, 1.0):
        p = oracle.params(1, 1, 1, kT=0.0, gamma_bulk=g, gamma_shear=g, gamma_odd=g, gamma_even=g)
        for _ in range(20):
            n = a * (1 + rng.normal(0, 0.3, 19))
            rho = n.sum()
            u = (n @ c) / rho
            neq = oracle.equilibrium(rho, u)
            np.testing.assert_allclose(oracle.collide_site(p, n, 0, 0), neq + g * (n - neq),
                                       atol=1e-15)


def test_equilibrium_is_deterministic_fixed_point(tabs):
    c, a, e, w = tabs
    p = oracle.params(5, 4, 3, kT=0.0, gamma_bulk=0.3, gamma_shear=-0.2, gamma_odd=0.6, gamma_even=0.1)
    u = np.array([0.02, -0.01, 0.03])
    fields = np.zeros((4, 3, 4, 5))
    fields[0] = 1.1
    fields[1:] = u[:, None, None, None]
    n0 = oracle.init(p, oracle.INIT_FIELDS, fields)
    n = oracle.run(p, n0, 0, 10)
    np.testing.assert_allclose(n, n0, atol=1e-15)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 5), (4, 3, 2), (7, 1, 1), (1, 1, 9)])
def test_pure_streaming_is_periodic_shift(tabs, dims):
    """All gamma = 1 and kT = 0 make the collision the identity, so one step
    of Eq. LBE shifts population i by +c_i with periodic wrap."""
    c, a, e, w = tabs
    nx, ny, nz = dims
    p = oracle.params(nx, ny, nz, kT=0.0, gamma_bulk=1, gamma_shear=1, gamma_odd=1, gamma_even=1)
    rng = np.random.default_rng(4)
    n0 = a[:, None, None, None] * (1 + rng.normal(0, 0.1, (19, nz, ny, nx)))
    n1, bad = oracle.step(p, n0, 0)
    assert bad == 0
    for i in range(19):
        want = np.roll(n0[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        np.testing.assert_allclose(n1[i], want, atol=1e-15)
    # lcm(nx, ny, nz) steps of pure streaming return the initial state
    T = np.lcm.reduce([nx, ny, nz])
    np.testing.assert_allclose(oracle.run(p, n0, 0, T), n0, atol=1e-15)


def _single_site_histories(p, nsites, T):
    """Evolve nsites independent single sites (1^3 boxes: streaming is the
    identity) from rest for T collisions; return modes (T+1, nsites, 19)."""
    c, a, e, w = oracle.tables()
    out = np.zeros((T + 1, nsites, 19))
    for s in range(nsites):
        n = a * p.rho0
        out[0, s] = e @ (n - a * p.rho0)
        for t in range(T):
            n = oracle.collide_site(p, n, s, t)
            out[t + 1, s] = e @ (n - a * p.rho0)
    return out


def test_single_site_ar1_law():
    """On one site the update of each non-conserved mode is an AR(1)
    process (Eqs. updaterule, FDT): starting from rest,
    E[m_k(t)^2] = (1 - gamma_k^2t) mu rho w_k, and the lag-1
    autocorrelation in the stationary regime is gamma_k."""
    c, a, e, w = oracle.tables()
    kT = 1e-4
    mu = 3 * kT
    gb, gs, go, ge = 0.5, 0.8, -0.4, 0.0
    p = oracle.params(1, 1, 1, kT=kT, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go,
                      gamma_even=ge, seed=77)
    N, T = 4000, 12
    m = _single_site_histories(p, N, T)
    g = th.mode_gammas(gb, gs, go, ge)
    # conserved modes never move
    assert np.abs(m[:, :, :4]).max() < 1e-13  # rounding only
    for k in range(4, 19):
        for t in (1, 2, 5, 12):
            want = (1 - g[k] ** (2 * t)) * mu * w[k]
            got = np.mean(m[t, :, k] ** 2)  # m^eq ~ 0 here (j = 0)
            se = want * np.sqrt(2.0 / N)
            assert abs(got - want) < 5 * se + 1e-12, (k, t, got, want)
        if g[k] != 0:
            x, y = m[6:-1, :, k].ravel(), m[7:, :, k].ravel()
            r = np.mean(x * y) / np.sqrt(np.mean(x * x) * np.mean(y * y))
            assert abs(r - g[k]) < 5 / np.sqrt(x.size), (k, r)


def test_random_stress_covariance_worked_example():
    """Sec. IV: one collision adds random stresses R with
    <R_xy^2> = mu rho cs^4 (1 - gs^2), <(R_yy - R_zz)^2> = 4 mu rho cs^4
    (1 - gs^2), <R_aa R_bb> = 6 mu rho cs^4 (1 - gb^2), and in general
    Eq. stressfluctuations_microscopic.  R = Pi*_neq - gamma Pi_neq is
    measured from populations with Pi_ab = sum_i n_i c_ia c_ib (Eq.
    defstress) on independent sites carrying a random non-equilibrium
    stress before the collision."""
    c, a, e, w = oracle.tables()
    kT, rho0 = 2e-4, 1.3
    mu = 3 * kT
    gb, gs = 0.3, 0.6
    p = oracle.params(1, 1, 1, rho0=rho0, kT=kT, gamma_bulk=gb, gamma_shear=gs,
                      gamma_odd=0.0, gamma_even=0.0, seed=5)
    rng = np.random.default_rng(6)
    N = 20000
    base = a * rho0
    R = np.zeros((N, 3, 3))
    for s in range(N):
        # a rest site (rho = rho0, j = 0) with random shear and bulk stress:
        # perturb along modes 4..9 only, so j stays 0 and m^eq stays 0
        dm = np.zeros(19)
        dm[4:10] = rng.normal(0, 1e-3, 6)
        n = base + a * (e.T @ (dm / w))
        Pi0 = np.einsum("i,ia,ib->ab", n - base, c, c)
        n1 = oracle.collide_site(p, n, s, 0)
        Pi1 = np.einsum("i,ia,ib->ab", n1 - base, c, c)
        tr0, tr1 = np.trace(Pi0), np.trace(Pi1)
        dev0 = Pi0 - tr0 / 3 * np.eye(3)
        dev1 = Pi1 - tr1 / 3 * np.eye(3)
        R[s] = (dev1 - gs * dev0) + (tr1 - gb * tr0) / 3 * np.eye(3)
    unit = mu * rho0 * CS2 ** 2
    golden = {}
    with open(th.os.path.join(th.GOLDEN, "stress_covariance.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, cs_, cb_ = line.split()
            golden[name] = float(cs_) * (1 - gs ** 2) + float(cb_) * (1 - gb ** 2)
    se = lambda v: 5 * v * np.sqrt(2.0 / N)
    v = np.mean(R[:, 0, 1] ** 2) / unit
    assert abs(v - golden["Rxy_Rxy"]) < se(golden["Rxy_Rxy"])
    v = np.mean((R[:, 1, 1] - R[:, 2, 2]) ** 2) / unit
    assert abs(v - golden["Ryy-Rzz_sq"]) < se(golden["Ryy-Rzz_sq"])
    tr = np.trace(R, axis1=1, axis2=2)
    v = np.mean(tr * tr) / unit
    assert abs(v - golden["trace_sq"]) < se(golden["trace_sq"])
    # general isotropic form, all 81 entries
    d = 3
    for al, be, ga, de in itertools.product(range(3), repeat=4):
        prod = R[:, al, be] * R[:, ga, de] / unit
        want = (1 - gs ** 2) * ((al == ga) * (be == de) + (al == de) * (be == ga)) \
            + 2.0 / d * (gs ** 2 - gb ** 2) * (al == be) * (ga == de)
        tol = 5 * prod.std() / np.sqrt(N)
        assert abs(prod.mean() - want) < tol, (al, be, ga, de, prod.mean(), want)


def test_negative_density_is_an_error(tabs):
    c, a, e, w = tabs
    p = oracle.params(1, 1, 1, kT=1e-4)
    with pytest.raises(ValueError):
        oracle.collide_site(p, -a, 0, 0)
    with pytest.raises(ValueError):
        oracle.collide_site(p, np.full(19, np.nan), 0, 0)
