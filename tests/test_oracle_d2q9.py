"""Pins of the oracle's D2Q9 lattice (Table I) against what the paper and the
mathematics fix, the two-dimensional counterparts of the D3Q19 pins:

* the velocity set and weights: normalisation and the isotropy conditions
  sigma_2 = c_s^2, sigma_4 = sigma_2^2, kappa_4 = 0 (Eqs. wi0-wi4,
  equilcond2-equilcond3), which fix the weights of a three-speed model;
* Table I's polynomials and printed lengths w_k, exact orthogonality, and the
  closed-form hydrodynamic vectors of Sec. III written for d = 2;
* the equilibrium's moments, conservation, the fixed point and pure
  streaming;
* the single-site AR(1) law (Sec. IV) and the random-stress covariance of
  Eq. stressfluctuations_microscopic at d = 2;
* the stationary law: mode variances mu rho w_k and a flat S(q);
* hydrodynamics: waves follow the linearised operator, whose q -> 0 limits
  are Eq. shearviscosity and Eq. bulkviscosity with d = 2, and the box-summed
  random stress has the covariance of Eq. macrostressfluct at d = 2."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import lbtheory as th

CS2 = 1.0 / 3.0
LAT = oracle.D2Q9
TABLE = "table1_d2q9.txt"


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables(LAT)


def p2(nx, ny, **kw):
    return oracle.params(nx, ny, 1, lattice=LAT, **kw)


def test_velocity_set_is_d2q9(tabs):
    c, a, e, w = tabs
    want = {(x, y, 0) for x, y in itertools.product((-1, 0, 1), repeat=2)}
    assert {tuple(map(int, v)) for v in c} == want
    for i in range(1, 9):
        o = i + 1 if i % 2 else i - 1
        assert tuple(-c[i]) == tuple(c[o])


def test_weights_fixed_by_isotropy_conditions(tabs):
    """Exact rationals: sum a = 1, odd moments vanish, sigma_2 = 1/3,
    sigma_4 = sigma_2^2, kappa_4 = 0; and these conditions have one solution
    (a0, a1, a2) for speeds 0, 1, sqrt 2 (solve the linear part, then the
    quadratic one)."""
    c, a, e, w = tabs
    aw = [Fraction(x).limit_denominator(1000) for x in a]
    assert all(float(f) == x for f, x in zip(aw, a))
    cv = [tuple(int(v) for v in ci[:2]) for ci in c]
    assert sum(aw) == 1
    cs2 = Fraction(1, 3)
    for al in range(2):
        assert sum(x * ci[al] for x, ci in zip(aw, cv)) == 0
        for be in range(2):
            assert sum(x * ci[al] * ci[be] for x, ci in zip(aw, cv)) == (cs2 if al == be else 0)
    for idx in itertools.product(range(2), repeat=4):
        al, be, ga, de = idx
        m4 = sum(x * ci[al] * ci[be] * ci[ga] * ci[de] for x, ci in zip(aw, cv))
        assert m4 == cs2 * cs2 * ((al == be) * (ga == de) + (al == ga) * (be == de) + (al == de) * (be == ga))
    # uniqueness: kappa_4 = 0 gives a1 = 4 a2; sigma_4 = sigma_2^2 gives
    # 4 a2 = (2 a1 + 4 a2)^2 = 144 a2^2, so a2 = 1/36 (a2 = 0 has no fourth
    # moment); then a1 and a0 follow
    a2 = Fraction(4, 144)
    assert (aw[5], aw[1], aw[0]) == (a2, 4 * a2, 1 - 16 * a2 - 4 * a2)


def test_table1_polynomials_lengths_and_orthogonality(tabs):
    c, a, e, w = tabs
    ex = th.table2_matrix(c, TABLE)
    rows = th.load_table2(TABLE)
    assert len(rows) == 9
    aw = [Fraction(x).limit_denominator(1000) for x in a]
    for k, _, wk in rows:
        for i in range(9):
            assert e[k, i] == float(ex[k][i])
        assert w[k] == pytest.approx(float(wk), rel=1e-15)
        assert sum(aw[i] * ex[k][i] ** 2 for i in range(9)) == wk
    for k, l in itertools.product(range(9), repeat=2):
        if k != l:
            assert sum(aw[i] * ex[k][i] * ex[l][i] for i in range(9)) == 0, (k, l)


def test_text_orthonormal_vectors_match_table1(tabs):
    """Sec. III's closed forms at d = 2: mass, momentum, bulk (k = d + 1),
    the diagonal shear vector (k = d + 2) and the off-diagonal one
    (k = 2d + 1) equal sqrt(a_i / w_k) e_ki of Table I."""
    c, a, e, w = tabs
    d = 2
    ehat = np.sqrt(a[None, :] / w[:, None]) * e
    cx, cy = c[:, 0].astype(float), c[:, 1].astype(float)
    c2 = cx ** 2 + cy ** 2
    sa = np.sqrt(a)
    text = {
        0: sa, 1: np.sqrt(a / CS2) * cx, 2: np.sqrt(a / CS2) * cy,
        3: (1 / CS2) * np.sqrt(a / (2 * d)) * (c2 - d * CS2),
        4: (1 / CS2) * np.sqrt(a / (2 * d * (d - 1))) * (d * cx ** 2 - c2),
        5: sa / CS2 * cx * cy,
    }
    for k, v in text.items():
        np.testing.assert_allclose(ehat[k], v, atol=1e-15, err_msg=f"mode {k}")
    np.testing.assert_allclose(ehat @ ehat.T, np.eye(9), atol=1e-14)
    np.testing.assert_allclose(ehat.T @ ehat, np.eye(9), atol=1e-14)


def test_equilibrium_moments(tabs):
    c, a, e, w = tabs
    cc = c[:, :2].astype(float)
    rng = np.random.default_rng(1)
    for _ in range(50):
        rho = rng.uniform(0.5, 2.0)
        u = rng.normal(0, 0.05, 2)
        neq = oracle.equilibrium(rho, [u[0], u[1], 0.0], LAT)
        assert neq.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(neq @ cc, rho * u, atol=1e-15)
        Pi = np.einsum("i,ia,ib->ab", neq, cc, cc)
        np.testing.assert_allclose(Pi, rho * CS2 * np.eye(2) + rho * np.outer(u, u), atol=1e-15)


def test_conservation_srt_and_fixed_point(tabs):
    c, a, e, w = tabs
    rng = np.random.default_rng(2)
    p = p2(1, 1, kT=1e-3, gamma_bulk=-0.3, gamma_shear=0.7, gamma_odd=0.2, gamma_even=-0.4, seed=11)
    for s in range(100):
        n = a * (1 + rng.normal(0, 0.2, 9))
        out = oracle.collide_site(p, n, s, s * 7)
        assert out.sum() == pytest.approx(n.sum(), rel=1e-14)
        np.testing.assert_allclose(out @ c, n @ c, atol=1e-15)
        assert not np.allclose(out, n)
    # single relaxation time: kT = 0 and one gamma for all modes
    for g in (0.0, 0.5, -0.8):
        p = p2(1, 1, gamma_bulk=g, gamma_shear=g, gamma_odd=g, gamma_even=g)
        n = a * (1 + rng.normal(0, 0.3, 9))
        rho = n.sum()
        neq = oracle.equilibrium(rho, (n @ c) / rho, LAT)
        np.testing.assert_allclose(oracle.collide_site(p, n, 0, 0), neq + g * (n - neq), atol=1e-15)
    # a uniform equilibrium is a fixed point of the deterministic update
    p = p2(5, 4, gamma_bulk=0.3, gamma_shear=-0.2, gamma_odd=0.6, gamma_even=0.1)
    f = np.zeros((3, 1, 4, 5))
    f[0], f[1], f[2] = 1.1, 0.02, -0.03
    n0 = oracle.init(p, oracle.INIT_FIELDS, f)
    np.testing.assert_allclose(oracle.run(p, n0, 0, 10), n0, atol=1e-15)


@pytest.mark.parametrize("dims", [(1, 1), (2, 2), (3, 5), (7, 1), (1, 6)])
def test_pure_streaming_is_periodic_shift(tabs, dims):
    c, a, e, w = tabs
    nx, ny = dims
    p = p2(nx, ny, gamma_bulk=1, gamma_shear=1, gamma_odd=1, gamma_even=1)
    rng = np.random.default_rng(4)
    n0 = a[:, None, None, None] * (1 + rng.normal(0, 0.1, (9, 1, ny, nx)))
    n1, bad = oracle.step(p, n0, 0)
    assert bad == 0
    for i in range(9):
        np.testing.assert_allclose(n1[i], np.roll(n0[i], shift=(c[i, 1], c[i, 0]), axis=(1, 2)), atol=1e-15)
    np.testing.assert_allclose(oracle.run(p, n0, 0, int(np.lcm(nx, ny))), n0, atol=1e-15)


def test_three_dimensional_box_rejected():
    p = oracle.params(4, 4, 2, lattice=LAT)
    with pytest.raises(ValueError):
        oracle.init(p, oracle.INIT_REST)
    buf = np.zeros(64)
    dp = oracle._dp(buf)
    assert oracle.lib().ora_equilibrium(7, 1.0, dp, dp) == -1


def test_single_site_ar1_law(tabs):
    """E[m_k(t)^2] = (1 - gamma_k^2t) mu rho w_k from rest, lag-1
    autocorrelation gamma_k (Eqs. updaterule, FDT)."""
    c, a, e, w = tabs
    kT = 1e-4
    mu = 3 * kT
    gb, gs, go, ge = 0.5, 0.8, -0.4, 0.3
    p = p2(1, 1, kT=kT, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go, gamma_even=ge, seed=77)
    N, T = 4000, 12
    m = np.zeros((T + 1, N, 9))
    for s in range(N):
        n = a.copy()
        for t in range(T):
            n = oracle.collide_site(p, n, s, t)
            m[t + 1, s] = e @ (n - a)
    g = th.mode_gammas(gb, gs, go, ge, q=9)
    assert np.abs(m[:, :, :3]).max() < 1e-13
    for k in range(3, 9):
        for t in (1, 2, 5, 12):
            want = (1 - g[k] ** (2 * t)) * mu * w[k]
            got = np.mean(m[t, :, k] ** 2)
            assert abs(got - want) < 5 * want * np.sqrt(2.0 / N) + 1e-12, (k, t, got, want)
        x, y = m[6:-1, :, k].ravel(), m[7:, :, k].ravel()
        r = np.mean(x * y) / np.sqrt(np.mean(x * x) * np.mean(y * y))
        assert abs(r - g[k]) < 5 / np.sqrt(x.size), (k, r)


def test_random_stress_covariance_microscopic(tabs):
    """Eq. stressfluctuations_microscopic at d = 2, in units of mu rho cs^4:
    <R_ab R_cd> = (1 - gs^2)(d_ac d_bd + d_ad d_bc) + (2/d)(gs^2 - gb^2) d_ab d_cd."""
    c, a, e, w = tabs
    kT, rho0, gb, gs = 2e-4, 1.3, 0.3, 0.6
    mu, d = 3 * kT, 2
    p = p2(1, 1, rho0=rho0, kT=kT, gamma_bulk=gb, gamma_shear=gs, seed=5)
    rng = np.random.default_rng(6)
    N = 20000
    cc = c[:, :2].astype(float)
    R = np.zeros((N, 2, 2))
    base = a * rho0
    for s in range(N):
        dm = np.zeros(9)
        dm[3:6] = rng.normal(0, 1e-3, 3)
        n = base + a * (e.T @ (dm / w))
        Pi0 = np.einsum("i,ia,ib->ab", n - base, cc, cc)
        Pi1 = np.einsum("i,ia,ib->ab", oracle.collide_site(p, n, s, 0) - base, cc, cc)
        tr0, tr1 = np.trace(Pi0), np.trace(Pi1)
        R[s] = (Pi1 - tr1 / d * np.eye(2) - gs * (Pi0 - tr0 / d * np.eye(2))) + (tr1 - gb * tr0) / d * np.eye(2)
    unit = mu * rho0 * CS2 ** 2
    for al, be, ga, de in itertools.product(range(2), repeat=4):
        prod = R[:, al, be] * R[:, ga, de] / unit
        want = (1 - gs ** 2) * ((al == ga) * (be == de) + (al == de) * (be == ga)) \
            + 2.0 / d * (gs ** 2 - gb ** 2) * (al == be) * (ga == de)
        assert abs(prod.mean() - want) < 5 * prod.std() / np.sqrt(N), (al, be, ga, de, prod.mean(), want)


def test_thermal_init_and_stationary_law(tabs):
    """Every mode's variance is mu rho0 w_k, from the thermal initial state
    and after many noisy steps; S(q) is flat at mu rho0."""
    c, a, e, w = tabs
    kT, rho0, L = 1e-4, 1.0, 32
    mu = 3 * kT
    p = p2(L, L, rho0=rho0, kT=kT, gamma_bulk=0.8, gamma_shear=-0.3, gamma_odd=0.4, gamma_even=-0.5,
           seed=4321)
    n = oracle.init(p, oracle.INIT_THERMAL)
    m = th.neq_modes_any(oracle.modes(p, n), rho0, c, a, e)
    for k in range(9):
        assert abs(m[k].var() / (mu * rho0 * w[k]) - 1) < 5 * np.sqrt(2.0 / L ** 2), k
    var, sq, t = [], [], 0
    for snap in range(200):
        n = oracle.run(p, n, t, 5)
        t += 5
        m = th.neq_modes_any(oracle.modes(p, n), rho0, c, a, e)
        var.append(m.reshape(9, -1).var(axis=1))
        sq.append(np.abs(np.fft.fft2(m[0, 0])) ** 2 / L ** 2)
    var = np.array(var)
    for k in range(9):
        r = var[:, k] / (mu * rho0 * w[k])
        b = np.array([x.mean() for x in np.array_split(r, 10)])
        se = b.std(ddof=1) / np.sqrt(10)
        assert abs(r.mean() - 1) < max(5 * se, 0.003) and abs(r.mean() - 1) < 0.02, (k, r.mean(), se)
    S = np.mean(sq, axis=0) / (mu * rho0)
    assert S[0, 0] < 1e-20
    kq = np.fft.fftfreq(L) * L
    kk = np.sqrt(kq[:, None] ** 2 + kq[None, :] ** 2)
    for lo, hi in [(0.5, 4), (4, 8), (8, 12), (12, 23)]:
        sel = (kk >= lo) & (kk < hi)
        assert abs(S[sel].mean() - 1) < 0.03, (lo, hi, S[sel].mean())


@pytest.mark.parametrize("kind", ["shear", "sound"])
def test_wave_follows_linear_operator(tabs, kind):
    """A kT = 0 wave along y on an 1 x L box evolves by diag(exp(-i q.c))
    Minv Gamma M built from Table I."""
    c, a, e, w = tabs
    L, nq, T, U = 32, 2, 60, 1e-6
    gb, gs, go, ge = -0.2, 0.9, 0.3, -0.6
    p = p2(1, L, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go, gamma_even=ge)
    y = np.arange(L)
    f = np.zeros((3, 1, L, 1))
    f[0] = 1.0
    if kind == "shear":
        f[1, 0, :, 0] = U * np.sin(2 * np.pi * nq * y / L)
    else:
        f[0, 0, :, 0] = 1.0 + U * np.sin(2 * np.pi * nq * y / L)
    n0 = oracle.init(p, oracle.INIT_FIELDS, f)
    nT = oracle.run(p, n0, 0, T)
    ph = np.exp(-2j * np.pi * nq * y / L)
    four = lambda n: (n[:, 0, :, 0] * ph[None, :]).sum(axis=1)
    Lop = th.one_step_operator([0, 2 * np.pi * nq / L, 0], th.mode_gammas(gb, gs, go, ge, q=9), c, a, e, w)
    want = np.linalg.matrix_power(Lop, T) @ four(n0)
    assert np.abs(four(nT) - want).max() < 1e-8 * np.abs(four(n0)).max()


@pytest.mark.parametrize("gs,gb", [(0.5, 0.5), (0.9, 0.0), (0.0, 0.7)])
def test_viscosities_closed_form(tabs, gs, gb):
    """q -> 0 limits: -ln|lambda_T| / q^2 -> nu of Eq. shearviscosity, the
    sound attenuation -> (2 nu (1 - 1/d) + zeta / rho) / 2 with zeta of Eq.
    bulkviscosity at d = 2, and the sound speed -> c_s."""
    c, a, e, w = tabs
    g = th.mode_gammas(gb, gs, 0.0, 0.0, q=9)
    L = 2048
    ns = np.array([1, 2, 4])
    qs = 2 * np.pi * ns / L
    nu_eff = np.array([-np.log(abs(th.shear_eigenvalue(L, n, g, c, a, e, w, axis=1))) for n in ns]) / qs ** 2
    assert th.extrapolate_q0(qs ** 2, nu_eff) == pytest.approx(th.nu_closed_form(gs), rel=1e-6)
    lam = np.array([th.sound_eigenvalue(L, n, g, c, a, e, w, axis=1) for n in ns])
    att = -np.log(np.abs(lam)) / qs ** 2
    want = 0.5 * (2 * th.nu_closed_form(gs) * (1 - 1 / 2) + th.zeta_closed_form(gb, d=2))
    assert th.extrapolate_q0(qs ** 2, att) == pytest.approx(want, rel=2e-3)
    assert th.extrapolate_q0(qs ** 2, np.abs(np.angle(lam)) / qs) == pytest.approx(np.sqrt(CS2), rel=1e-4)


def test_macroscopic_random_stress_covariance(tabs):
    """Eq. macrostressfluct at d = 2 for the box-summed random stress of a
    full run with streaming (see the D3Q19 version)."""
    c, a, e, w = tabs
    L, rho0, kT, gb, gs = 3, 1.3, 1e-4, 0.3, 0.5
    p = p2(L, L, rho0=rho0, kT=kT, gamma_bulk=gb, gamma_shear=gs, gamma_odd=0.4, gamma_even=-0.3, seed=8)
    g = th.mode_gammas(gb, gs, 0.4, -0.3, q=9)
    n = oracle.init(p, oracle.INIT_THERMAL)
    N, T = L * L, 20000
    m = oracle.modes(p, n)
    rho_bar = rho0 + m[0].mean()
    Q = np.empty((T, 2, 2))
    for t in range(T):
        n = oracle.run(p, n, t, 1)
        m1 = oracle.modes(p, n)
        Q[t] = th.macroscopic_stress(th.box_random_stress(m, m1, rho0, g, c, a, e, w), gb, gs, d=2)
        m = m1
    eta = rho_bar * th.nu_closed_form(gs)
    zeta = rho_bar * th.zeta_closed_form(gb, d=2)
    want = N * th.macro_stress_covariance(kT, eta, zeta, d=2)
    for idx in itertools.product(range(2), repeat=4):
        al, be, ga, de = idx
        prod = Q[:, al, be] * Q[:, ga, de]
        tol = 5 * prod.std() / np.sqrt(T) + 1e-3 * abs(want[idx])
        assert abs(prod.mean() - want[idx]) < tol, (idx, prod.mean(), want[idx])
