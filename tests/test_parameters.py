"""Parameter choice (Sec. VI): the mapping from physical spacing, time step,
density, viscosities and temperature to lattice parameters must reproduce
the physical viscosities through the Chapman-Enskog results of Sec. V
(Eqs. shearviscosity, bulkviscosity) and the fluctuation level through
mu = k_B T h^2 / (c_s_hat^2 b^(d+2)) with k_B T = m_p c_s^2 (Eq. mpeos)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_0707_1581_amd import lb
from tests import lbtheory as th

# water-like fluid at a nanometre lattice spacing, SI units
WATER = dict(b=1e-9, h=1e-12, rho=1000.0, eta=8.9e-4, zeta=2.5e-3, kBT=1.380649e-23 * 300)


def test_viscosities_round_trip_through_chapman_enskog():
    for case in (WATER, dict(WATER, h=5e-13, b=2e-9), dict(b=1.0, h=1.0, rho=1.0, eta=0.5 / 3, zeta=0.2, kBT=1e-4)):
        q = lb.physical_params(**case)
        b, h, rho = case["b"], case["h"], case["rho"]
        # Eq. shearviscosity in lattice units (h = 1, c_s^2 = 1/3, rho0 = 1), back to physical units
        nu_lat = th.nu_closed_form(q["gamma_shear"])
        assert nu_lat * b * b / h == pytest.approx(case["eta"] / rho, rel=1e-12)
        zeta_lat = th.zeta_closed_form(q["gamma_bulk"])
        assert zeta_lat * b * b / h == pytest.approx(case["zeta"] / rho, rel=1e-12)
        assert -1 < q["gamma_shear"] < 1 and -1 < q["gamma_bulk"] < 1
        assert q["rho0"] == 1.0


def test_temperature_maps_to_fluctuation_level():
    """Sec. VI: mu = k_B T h^2 / (c_s_hat^2 b^(d+2)); in lattice units (mass
    unit rho b^3) the density variance per site mu_lattice * rho0 must equal
    the physical relative density variance k_B T / (rho c_s^2 b^3) (ideal-gas
    compressibility with k_B T = m_p c_s^2, Eq. mpeos)."""
    q = lb.physical_params(**WATER)
    b, h, rho, kBT = WATER["b"], WATER["h"], WATER["rho"], WATER["kBT"]
    cs2 = (1.0 / 3.0) * b * b / (h * h)
    mu_lat = 3.0 * q["kT"]
    assert mu_lat == pytest.approx(kBT / (rho * cs2 * b ** 3), rel=1e-12)


def test_mapped_lattice_decays_at_physical_viscosity():
    """A shear wave on the mapped lattice (oracle, 1 x 1 x 1024, long wave)
    decays at the physical eta / rho once converted back to SI units."""
    q = lb.physical_params(**dict(WATER, h=2e-13))
    c, a, e, w = oracle.tables()
    L = 1024
    lam = abs(th.shear_eigenvalue(L, 1, th.mode_gammas(q["gamma_bulk"], q["gamma_shear"], 0, 0), c, a, e, w))
    k = 2 * np.pi / L
    nu_lat = -np.log(lam) / k ** 2
    b, h = WATER["b"], 2e-13
    assert nu_lat * b * b / h == pytest.approx(WATER["eta"] / WATER["rho"], rel=1e-3)


@pytest.mark.parametrize("bad", [dict(b=0.0), dict(h=-1.0), dict(rho=float("nan")), dict(eta=0.0),
                                 dict(zeta=-2.0), dict(kBT=-1.0)])
def test_invalid_physical_parameters(bad):
    args = dict(WATER, **bad)
    p = lb.make_params(4, 4, 4, kT=7.0)
    rc = lb.lib().lb_params_from_physical(args["b"], args["h"], args["rho"], args["eta"], args["zeta"],
                                           args["kBT"], ctypes.byref(p))
    assert rc == lb.LB_EINVAL
    assert p.kT == 7.0


def test_two_dimensional_mapping():
    """D2Q9 (d = 2): rho is a mass per area, mu = k_B T h^2 / (c_s_hat^2 b^4),
    zeta of Eq. bulkviscosity carries 1/d = 1/2; the mapped shear and sound
    waves of the D2Q9 linear operator decay at the physical viscosities."""
    case = dict(b=1e-9, h=2e-13, rho=1e-6, eta=8.9e-13, zeta=2.5e-12, kBT=1.380649e-23 * 300)
    q = lb.physical_params(**case, lattice="d2q9")
    b, h, rho = case["b"], case["h"], case["rho"]
    assert th.nu_closed_form(q["gamma_shear"]) * b * b / h == pytest.approx(case["eta"] / rho, rel=1e-12)
    assert th.zeta_closed_form(q["gamma_bulk"], d=2) * b * b / h == pytest.approx(case["zeta"] / rho, rel=1e-12)
    cs2 = (1.0 / 3.0) * b * b / (h * h)
    assert 3.0 * q["kT"] == pytest.approx(case["kBT"] / (rho * cs2 * b ** 2), rel=1e-12)
    # the 3D mapping of the same numbers differs (d enters gamma_bulk and mu)
    q3 = lb.physical_params(**case)
    assert q3["gamma_bulk"] != pytest.approx(q["gamma_bulk"]) and q3["kT"] != pytest.approx(q["kT"])
    c, a, e, w = oracle.tables(oracle.D2Q9)
    g = th.mode_gammas(q["gamma_bulk"], q["gamma_shear"], 0, 0, q=9)
    L = 1024
    k = 2 * np.pi / L
    nu_lat = -np.log(abs(th.shear_eigenvalue(L, 1, g, c, a, e, w, axis=1))) / k ** 2
    assert nu_lat * b * b / h == pytest.approx(case["eta"] / rho, rel=1e-3)
    att = -np.log(abs(th.sound_eigenvalue(L, 1, g, c, a, e, w, axis=1))) / k ** 2
    want = 0.5 * (case["eta"] + case["zeta"]) / rho  # (2 eta (1 - 1/d) + zeta) / (2 rho) at d = 2
    assert att * b * b / h == pytest.approx(want, rel=3e-3)
