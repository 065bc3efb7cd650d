"""Pins of the oracle's stress-only branch (thermal_modes = 1): the earlier
model the paper contrasts with its detailed-balance collision, in which only
the stress modes (bulk and shear) receive noise and the kinetic modes relax
without any (Sec. I on the earlier model, Sec. IV on the degrees of freedom
that must be thermalised for detailed balance).

What the paper and the mathematics fix for that model:
  - one collision leaves the conserved modes alone, gives the stress modes
    exactly what the detailed-balance collision gives them (the same normals
    in the same places, Eq. FDT), and turns each kinetic mode into
    gamma_k m_k with nothing added (no equilibrium part, Sec. V, and no
    noise);
  - on one site (1^3 box, streaming the identity) the stress modes follow
    the AR(1) law of Eqs. updaterule / FDT, E[m_k^2(t)] = (1 - gamma_k^2t)
    mu rho w_k from rest, while the kinetic modes stay exactly zero from
    rest and decay as gamma_k^t from any start, independent of the seed;
  - with streaming, the stationary state is the one of the linearised
    update with noise on the stress modes only (a discrete Lyapunov
    equation per wave vector, solved independently in tests/lbtheory.py):
    every mode, the stress modes included, sits well below mu rho w_k at
    the lattice scale, while long density waves keep the hydrodynamic value
    S(q -> 0) = mu rho.
A slip such as the bulk mode dropped from the noisy set, kinetic modes still
noised, or the normals shifted by one mode fails one of these."""
import numpy as np
import pytest

import oracle
from tests import lbtheory as th

KT = 1e-4
MU = 3 * KT


def _perturbed_site(a, e, w, rho0, rng, scale=1e-3):
    """Populations of one site with every mode, kinetic ones included,
    displaced from rest."""
    dm = rng.normal(0, scale, len(w))
    return a * rho0 + a * (e.T @ (dm / w))


@pytest.mark.parametrize("lattice", [oracle.D3Q19, oracle.D2Q9])
def test_one_collision_stress_only_against_detailed_balance(lattice):
    c, a, e, w = oracle.tables(lattice)
    q = len(a)
    d = 3 if lattice == oracle.D3Q19 else 2
    nstress = 6 if d == 3 else 3
    go, ge = -0.4, 0.3
    g = th.mode_gammas(0.3, 0.7, go, ge, q)
    kw = dict(rho0=1.2, kT=KT, gamma_bulk=0.3, gamma_shear=0.7, gamma_odd=go, gamma_even=ge, seed=99,
              lattice=lattice)
    p_all = oracle.params(1, 1, 1, thermal_modes=oracle.THERMAL_ALL, **kw)
    p_st = oracle.params(1, 1, 1, thermal_modes=oracle.THERMAL_STRESS_ONLY, **kw)
    rng = np.random.default_rng(3)
    kin = slice(d + 1 + nstress, q)
    noise_seen = 0.0
    for site, t in [(0, 0), (5, 17), (2 ** 32 - 1, 2 ** 33 + 5)]:
        n = _perturbed_site(a, e, w, 1.2, rng)
        m = e @ n
        ma = e @ oracle.collide_site(p_all, n, site, t)
        ms = e @ oracle.collide_site(p_st, n, site, t)
        scale = np.sqrt(MU * 1.2 * w)
        # conserved modes untouched by both
        np.testing.assert_allclose(ms[:d + 1], m[:d + 1], rtol=0, atol=1e-14)
        # stress modes: identical to the detailed-balance collision (same normals, same amplitudes)
        np.testing.assert_allclose(ms[d + 1:d + 1 + nstress], ma[d + 1:d + 1 + nstress], rtol=0,
                                   atol=1e-14 * scale.max())
        # and they did receive noise: the noiseless collision (kT = 0) differs by O(sqrt(mu))
        p0 = oracle.params(1, 1, 1, thermal_modes=oracle.THERMAL_STRESS_ONLY, **dict(kw, kT=0.0))
        md = e @ oracle.collide_site(p0, n, site, t)
        assert np.abs((ms - md)[d + 1:d + 1 + nstress] / scale[d + 1:d + 1 + nstress]).max() > 0.05
        # kinetic modes: relaxed by gamma_k with nothing added
        np.testing.assert_allclose(ms[kin], g[kin] * m[kin], rtol=0, atol=1e-15)
        # the detailed-balance collision does add noise there, of the right size
        noise_seen = max(noise_seen, float(np.abs((ma[kin] - g[kin] * m[kin]) / scale[kin]).max()))
    assert noise_seen > 0.1


def _site_histories(p, lattice, nsites, T, start=None):
    c, a, e, w = oracle.tables(lattice)
    q = len(a)
    out = np.zeros((T + 1, nsites, q))
    for s in range(nsites):
        n = a * p.rho0 if start is None else start(s)
        out[0, s] = e @ (n - a * p.rho0)
        for t in range(T):
            n = oracle.collide_site(p, n, s, t)
            out[t + 1, s] = e @ (n - a * p.rho0)
    return out


def test_single_site_stress_only_ar1_law():
    """1^3 box: the stress modes are AR(1) with variance (1 - gamma^2t)
    mu rho w_k from rest and lag-1 correlation gamma_k; the kinetic modes
    stay at zero (rounding) whatever their rates."""
    c, a, e, w = oracle.tables()
    gb, gs, go, ge = 0.5, 0.8, -0.4, 0.6
    p = oracle.params(1, 1, 1, kT=KT, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go, gamma_even=ge,
                      seed=77, thermal_modes=oracle.THERMAL_STRESS_ONLY)
    N, T = 4000, 12
    m = _site_histories(p, oracle.D3Q19, N, T)
    g = th.mode_gammas(gb, gs, go, ge)
    assert np.abs(m[:, :, :4]).max() < 1e-13
    assert np.abs(m[:, :, 10:]).max() < 1e-13  # rounding only; noise would be ~1e-2
    for k in range(4, 10):
        for t in (1, 2, 5, 12):
            want = (1 - g[k] ** (2 * t)) * MU * w[k]
            got = np.mean(m[t, :, k] ** 2)
            assert abs(got - want) < 5 * want * np.sqrt(2.0 / N), (k, t, got, want)
        x, y = m[6:-1, :, k].ravel(), m[7:, :, k].ravel()
        r = np.mean(x * y) / np.sqrt(np.mean(x * x) * np.mean(y * y))
        assert abs(r - g[k]) < 5 / np.sqrt(x.size), (k, r)


def test_single_site_stress_only_kinetic_decay_is_deterministic():
    """From a start with displaced kinetic modes, m_k(t) = gamma_k^t m_k(0)
    for every kinetic mode, the same for every seed."""
    c, a, e, w = oracle.tables()
    go, ge = -0.4, 0.6
    g = th.mode_gammas(0.5, 0.8, go, ge)
    rng = np.random.default_rng(8)
    starts = [_perturbed_site(a, e, w, 1.0, rng) for _ in range(5)]
    hist = []
    for seed in (1, 2):
        p = oracle.params(1, 1, 1, kT=KT, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=go, gamma_even=ge,
                          seed=seed, thermal_modes=oracle.THERMAL_STRESS_ONLY)
        hist.append(_site_histories(p, oracle.D3Q19, 5, 8, start=lambda s: starts[s]))
    for h in hist:
        for t in range(9):
            np.testing.assert_allclose(h[t, :, 10:], (g[10:] ** t) * h[0, :, 10:], rtol=0, atol=1e-15)
    np.testing.assert_allclose(hist[0][:, :, 10:], hist[1][:, :, 10:], rtol=0, atol=1e-14)  # rounding only
    assert np.abs(hist[0][1:, :, 4:10] - hist[1][1:, :, 4:10]).max() > 1e-4 * np.sqrt(MU)


def _stationary_ratios(p, lattice, nsnap, every, burn):
    """Per-snapshot variances of m_k - m_k^eq (conserved modes about their
    lattice mean) over the box, divided by mu rho0 w_k."""
    c, a, e, w = oracle.tables(lattice)
    n = oracle.init(p, oracle.INIT_THERMAL)
    n = oracle.run(p, n, 0, burn)
    t = burn
    var = []
    for _ in range(nsnap):
        n = oracle.run(p, n, t, every)
        t += every
        m = th.neq_modes_any(oracle.modes(p, n), p.rho0, c, a, e)
        var.append(m.reshape(len(w), -1).var(axis=1) / (MU * p.rho0 * w))
    return np.array(var)


@pytest.mark.parametrize("lattice,dims,gb,gs", [(oracle.D3Q19, (8, 8, 8), 0.5, 0.5),
                                                (oracle.D3Q19, (8, 8, 8), 0.2, 0.8),
                                                (oracle.D2Q9, (24, 24, 1), 0.5, 0.5)])
def test_stress_only_stationary_law_matches_linear_theory(lattice, dims, gb, gs):
    c, a, e, w = oracle.tables(lattice)
    q = len(a)
    d = 3 if lattice == oracle.D3Q19 else 2
    g = th.mode_gammas(gb, gs, 0.0, 0.0, q)
    noisy = np.zeros(q, bool)
    noisy[d + 1:d + 1 + (6 if d == 3 else 3)] = True
    want = th.stationary_mode_variances(dims, g, noisy, c, a, e, w)
    # the contrast: the same rates with noise on every non-conserved mode give mu rho w_k
    full = noisy.copy()
    full[d + 1:] = True
    ones = th.stationary_mode_variances(dims, g, full, c, a, e, w)
    np.testing.assert_allclose(ones[d + 1:], 1.0, atol=1e-9)
    assert want.max() < 0.75  # every mode under-thermalised at the lattice scale
    p = oracle.params(*dims, kT=KT, gamma_bulk=gb, gamma_shear=gs, seed=2024, lattice=lattice,
                      thermal_modes=oracle.THERMAL_STRESS_ONLY)
    var = _stationary_ratios(p, lattice, nsnap=400, every=5, burn=200)
    blocks = np.array([b.mean(axis=0) for b in np.array_split(var, 10)])
    got = var.mean(axis=0)
    se = blocks.std(axis=0, ddof=1) / np.sqrt(len(blocks))
    for k in range(q):
        assert abs(got[k] - want[k]) < max(5 * se[k], 0.01 * want[k]), (k, got[k], want[k], se[k])
        assert abs(got[k] / want[k] - 1) < 0.03, (k, got[k], want[k])


def test_stress_only_long_waves_keep_hydrodynamic_density_fluctuations():
    """Linear theory of both models: the detailed-balance collision has
    S(q) = mu rho at every wave vector (Eq. mpeos); in the stress-only model
    the deficit 1 - S(q) vanishes like q^2 towards the longest waves (the
    hydrodynamic limit is right) and is large at short ones."""
    c, a, e, w = oracle.tables()
    g = th.mode_gammas(0.5, 0.5, 0.0, 0.0)
    noisy = np.zeros(19, bool)
    noisy[4:10] = True
    full = noisy.copy()
    full[4:] = True
    _, sq_full = th.stationary_mode_variances((16, 16, 16), g, full, c, a, e, w, structure_factor=True)
    np.testing.assert_allclose(list(sq_full.values()), 1.0, atol=1e-9)
    deficit = {}
    for L in (16, 32):
        _, sq = th.stationary_mode_variances((L, L, L), g, noisy, c, a, e, w, structure_factor=True)
        k1 = (2 * np.pi / L) ** 2
        shell = {int(round(k2 / k1)): v for k2, v in sq.items()}
        deficit[L] = 1 - shell[2]  # the (1, 1, 0) shell
        short = [v for k2, v in sq.items() if k2 > 2.0]
        assert np.mean(short) < 0.7, (L, np.mean(short))
    assert deficit[16] > 0.1
    # q^2 four times smaller: deficit about four times smaller (O(q^2) plus O(q^4))
    assert 0.2 < deficit[32] / deficit[16] < 0.35, deficit
