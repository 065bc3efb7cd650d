"""Stationary-law pins of the oracle.

The single-site Gaussian law of Eq. probdistfluct2 / Eq. modeprob with the
scaling of Eqs. xdef and evectors_orthonormal gives, for every
non-conserved mode, <(m_k - m_k^eq)^2> = mu rho w_k (unscaled modes
m_k = sum_i e_ki n_i).  Because streaming only permutes populations, the
product of these laws over sites is stationary, so conserved modes
fluctuate about their lattice mean with the same variance: density variance
mu rho = rho kT / c_s^2 with a flat structure factor, and momentum variance
rho kT per component (Eq. mpeos, k_B T = m_p c_s^2)."""
import numpy as np
import pytest

import oracle
from tests import lbtheory as th


def _batched_ratio(samples, want, nbatch=10):
    """mean ratio and its standard error from batch means (samples along
    axis 0 are snapshots, each already a per-snapshot variance)."""
    r = np.asarray(samples) / want
    b = np.array_split(r, nbatch)
    means = np.array([x.mean() for x in b])
    return r.mean(), means.std(ddof=1) / np.sqrt(nbatch)


def test_thermal_init_samples_stationary_law():
    c, a, e, w = oracle.tables()
    kT, rho0 = 1e-4, 1.0
    mu = 3 * kT
    p = oracle.params(32, 32, 32, rho0=rho0, kT=kT, seed=1234)
    n = oracle.init(p, oracle.INIT_THERMAL)
    m = th.neq_modes(oracle.modes(p, n), rho0)
    N = 32 ** 3
    for k in range(19):
        ratio = m[k].var() / (mu * rho0 * w[k])
        assert abs(ratio - 1) < 5 * np.sqrt(2.0 / N), (k, ratio)


@pytest.mark.parametrize("gs,gb,go,ge", [(0.5, 0.5, 0.0, 0.0), (0.8, -0.3, 0.4, -0.5)])
def test_mode_variances_and_structure_factor(gs, gb, go, ge):
    c, a, e, w = oracle.tables()
    kT, rho0 = 1e-4, 1.0
    mu = 3 * kT
    L = 16
    p = oracle.params(L, L, L, rho0=rho0, kT=kT, gamma_bulk=gb, gamma_shear=gs,
                      gamma_odd=go, gamma_even=ge, seed=4321)
    n = oracle.init(p, oracle.INIT_THERMAL)
    var = []
    sq = []
    t = 0
    for snap in range(160):
        n = oracle.run(p, n, t, 5)
        t += 5
        m = th.neq_modes(oracle.modes(p, n), rho0)
        var.append(m.reshape(19, -1).var(axis=1))
        drho = m[0]
        sq.append(np.abs(np.fft.fftn(drho)) ** 2 / drho.size)
    var = np.array(var)
    for k in range(19):
        r, se = _batched_ratio(var[:, k], mu * rho0 * w[k])
        assert abs(r - 1) < max(5 * se, 0.003) and abs(r - 1) < 0.02, (k, r, se)
    # flat structure factor S(q) = mu rho0 for q != 0, radially binned
    S = np.mean(sq, axis=0) / (mu * rho0)
    assert S[0, 0, 0] < 1e-20  # S(0) = 0: total mass is exactly conserved
    k = np.fft.fftfreq(L) * L
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    for lo, hi in [(0.5, 3), (3, 6), (6, 9), (9, 15)]:
        sel = (kk >= lo) & (kk < hi)
        assert abs(S[sel].mean() - 1) < 0.03, (lo, hi, S[sel].mean())
