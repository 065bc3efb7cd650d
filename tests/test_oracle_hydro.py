"""Pins of the oracle on whole lattices.

* Deterministic waves (kT = 0) on 1 x 1 x L boxes evolve exactly by the
  linearised one-step operator diag(exp(-i q.c_i)) Minv Gamma M built from
  Table II (the quadratic equilibrium terms only feed other harmonics).
* The q -> 0 limits of that operator's shear and sound eigenvalues give the
  paper's closed forms: kinematic shear viscosity c_s^2 (1 + g_s) /
  (2 (1 - g_s)) (Eq. shearviscosity), bulk viscosity c_s^2 (1 + g_b) /
  (3 (1 - g_b)) (Eq. bulkviscosity) through the sound attenuation
  (4 nu / 3 + zeta / rho) / 2 of the linearised Eq. ce12, and the sound
  speed c_s = 1/sqrt(3) of the equation of state p = rho c_s^2 (Sec. II).
"""
import itertools

import numpy as np
import pytest

import oracle
from tests import lbtheory as th

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def _fourier(n, q_index, L):
    z = np.arange(L)
    return (n[:, :, 0, 0] * np.exp(-2j * np.pi * q_index * z / L)[None, :]).sum(axis=1)


@pytest.mark.parametrize("kind", ["shear", "sound"])
@pytest.mark.parametrize("gs,gb,go,ge", [(0.5, 0.5, 0.0, 0.0), (0.9, -0.2, 0.3, -0.6), (-0.5, 0.8, 0.0, 0.0)])
def test_wave_follows_linear_operator(tabs, kind, gs, gb, go, ge):
    c, a, e, w = tabs
    L, nq, T, U = 32, 2, 60, 1e-6
    p = oracle.params(1, 1, L, kT=0.0, gamma_bulk=gb, gamma_shear=gs, gamma_odd=go, gamma_even=ge)
    z = np.arange(L)
    fields = np.zeros((4, L, 1, 1))
    fields[0] = 1.0
    if kind == "shear":
        fields[1, :, 0, 0] = U * np.sin(2 * np.pi * nq * z / L)
    else:
        fields[0, :, 0, 0] = 1.0 + U * np.sin(2 * np.pi * nq * z / L)
    n0 = oracle.init(p, oracle.INIT_FIELDS, fields)
    nT = oracle.run(p, n0, 0, T)
    Lop = th.one_step_operator([0, 0, 2 * np.pi * nq / L], th.mode_gammas(gb, gs, go, ge), c, a, e, w)
    f0 = _fourier(n0, nq, L)
    want = np.linalg.matrix_power(Lop, T) @ f0
    got = _fourier(nT, nq, L)
    assert np.abs(got - want).max() < 1e-8 * np.abs(f0).max()


@pytest.mark.parametrize("gs", [0.0, 0.5, 0.8, 0.9])
def test_shear_viscosity_closed_form(tabs, gs):
    """Eq. shearviscosity: -ln|lambda_T(q)| / q^2 -> c_s^2 (1+g)/(2(1-g))."""
    c, a, e, w = tabs
    g = th.mode_gammas(0.5, gs, 0.0, 0.0)
    L = 2048  # long waves, where the O(q^2) lattice corrections are small
    ns = np.array([1, 2, 4])
    qs = 2 * np.pi * ns / L
    nu_eff = np.array([-np.log(abs(th.shear_eigenvalue(L, n, g, c, a, e, w))) for n in ns]) / qs ** 2
    nu0 = th.extrapolate_q0(qs ** 2, nu_eff)
    assert nu0 == pytest.approx(th.nu_closed_form(gs), rel=1e-6)


@pytest.mark.parametrize("gs,gb", [(0.5, 0.5), (0.8, 0.0), (0.0, 0.7)])
def test_sound_attenuation_and_speed(tabs, gs, gb):
    """Sound eigenvalue: |lambda| -> exp(-(4 nu/3 + zeta/rho)/2 q^2) with
    zeta from Eq. bulkviscosity, and phase -> c_s q with c_s^2 = 1/3."""
    c, a, e, w = tabs
    g = th.mode_gammas(gb, gs, 0.0, 0.0)
    L = 2048
    ns = np.array([1, 2, 4])
    qs = 2 * np.pi * ns / L
    lam = np.array([th.sound_eigenvalue(L, n, g, c, a, e, w) for n in ns])
    att = -np.log(np.abs(lam)) / qs ** 2
    want = 0.5 * (4.0 / 3.0 * th.nu_closed_form(gs) + th.zeta_closed_form(gb))
    assert th.extrapolate_q0(qs ** 2, att) == pytest.approx(want, rel=2e-3)
    speed = np.abs(np.angle(lam)) / qs
    assert th.extrapolate_q0(qs ** 2, speed) == pytest.approx(np.sqrt(CS2), rel=1e-4)


def test_shear_wave_decay_matches_eigenvalue_1x1xL(tabs):
    """Per-step decay of the j_x amplitude of a 1 x 1 x 128 shear wave
    (after the initial transient) equals |lambda_T(q)| to 1e-10."""
    c, a, e, w = tabs
    L, gs = 128, 0.9
    p = oracle.params(1, 1, L, kT=0.0, gamma_bulk=0.5, gamma_shear=gs)
    z = np.arange(L)
    fields = np.zeros((4, L, 1, 1))
    fields[0] = 1.0
    fields[1, :, 0, 0] = 1e-3 * np.sin(2 * np.pi * z / L)
    n = oracle.init(p, oracle.INIT_FIELDS, fields)
    n = oracle.run(p, n, 0, 200)
    amps = []
    for t in range(3):
        mom = oracle.moments(p, n)
        amps.append((2.0 / L) * (mom[1, :, 0, 0] * np.sin(2 * np.pi * z / L)).sum())
        n = oracle.run(p, n, 200 + t, 1)
    lam = abs(th.shear_eigenvalue(L, 1, th.mode_gammas(0.5, gs, 0, 0), c, a, e, w))
    assert amps[1] / amps[0] == pytest.approx(lam, abs=1e-10)
    assert amps[2] / amps[1] == pytest.approx(lam, abs=1e-10)


def test_macroscopic_random_stress_covariance():
    """Sec. V: the random stress Q on the hydrodynamic level, summed over a
    periodic box and measured from consecutive steps of a full run with
    streaming, has the Landau-Lifshitz covariance of Eq. macrostressfluct
    with the viscosities of Eqs. shearviscosity and bulkviscosity, N times
    the per-site value (sites are independent)."""
    L, rho0, kT, gb, gs = 3, 1.3, 1e-4, 0.3, 0.5
    p = oracle.params(L, L, L, rho0=rho0, kT=kT, gamma_bulk=gb, gamma_shear=gs,
                      gamma_odd=0.4, gamma_even=-0.3, seed=8)
    n = oracle.init(p, oracle.INIT_THERMAL)
    N, T = L ** 3, 20000
    c, a, e, w = oracle.tables()
    g = th.mode_gammas(gb, gs, 0.4, -0.3)
    rho_bar = rho0 + oracle.modes(p, n)[0].mean()
    Q = np.empty((T, 3, 3))
    m = oracle.modes(p, n)
    for t in range(T):
        n = oracle.run(p, n, t, 1)
        m1 = oracle.modes(p, n)
        Q[t] = th.macroscopic_stress(th.box_random_stress(m, m1, rho0, g, c, a, e, w), gb, gs)
        m = m1
    eta = rho_bar * th.nu_closed_form(gs)
    zeta = rho_bar * th.zeta_closed_form(gb)
    want = N * th.macro_stress_covariance(kT, eta, zeta)
    assert np.abs(Q.mean(axis=0)).max() < 5 * Q.std(axis=0).max() / np.sqrt(T)
    for idx in itertools.product(range(3), repeat=4):
        a, b, c, d = idx
        prod = Q[:, a, b] * Q[:, c, d]
        tol = 5 * prod.std() / np.sqrt(T) + 1e-3 * abs(want[idx])
        assert abs(prod.mean() - want[idx]) < tol, (idx, prod.mean(), want[idx])
    # the worked components: shear, normal, and normal-normal cross terms
    for (a, b, c, d), w in [((0, 1, 0, 1), 2 * kT * eta), ((0, 0, 0, 0), 2 * kT * (zeta + 4 * eta / 3)),
                            ((1, 1, 2, 2), 2 * kT * (zeta - 2 * eta / 3))]:
        assert want[a, b, c, d] == pytest.approx(N * w, rel=1e-12)
