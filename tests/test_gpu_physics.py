"""Physics of the GPU path at full size, against what the paper fixes.

* Stationary statistics (Eq. modeprob with Eqs. xdef and
  evectors_orthonormal): every mode's variance about equilibrium is
  mu rho w_k, so the density variance is rho kT / c_s^2 with a flat
  structure factor and the momentum variance rho kT (Eq. mpeos); checked on
  128^3 boxes to 1%.
* Deterministic shear waves on 128^3 boxes do not depend on x and y, so the
  box reduces exactly to a 1 x 1 x 128 lattice: the GPU's x,y-averaged j_x
  must follow the FP64 oracle's 1 x 1 x 128 run, and the decay rate must
  give the kinematic viscosity c_s^2 (1 + g_s) / (2 (1 - g_s)) of Eq.
  shearviscosity (after removing the O(q^2) lattice correction).
* The earlier model with noise on the stress modes only (Sec. IV) leaves the
  kinetic modes under-thermalised, and through streaming every other mode
  too: all 19 variances follow the linear theory of that model, well short
  of mu rho w_k.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_0707_1581_amd as lbf
import workloads
from tests import lbtheory as th
from tests.gpu_util import oracle_params, say

pytestmark = pytest.mark.gpu
W = np.array([36, 12, 12, 12, 24, 48, 16, 4, 4, 4, 24, 24, 24, 8, 8, 8, 72, 48, 16]) / 36.0


def neq_variances(modes, rho0):
    """Per-mode variance of the non-equilibrium part (conserved modes about
    their lattice mean) and the lattice-mean density, on the GPU in fp64."""
    m = modes.double()
    rho = rho0 + m[0]
    jx, jy, jz = m[1], m[2], m[3]
    eq = {4: (jx * jx + jy * jy + jz * jz) / rho, 5: (2 * jx * jx - jy * jy - jz * jz) / rho,
          6: (jy * jy - jz * jz) / rho, 7: jx * jy / rho, 8: jy * jz / rho, 9: jz * jx / rho}
    out = np.zeros(19)
    for k in range(19):
        x = m[k] - eq[k] if k in eq else m[k]
        x = x - x.mean() if k < 4 else x
        out[k] = float((x * x).mean())
    return out, float(rho.mean())


def structure_factor(m0):
    d = m0.double()
    d = d - d.mean()
    f = torch.fft.fftn(d)
    return (f.real ** 2 + f.imag ** 2) / d.numel()


@pytest.mark.parametrize("gs", [0.0, 0.5, 0.9])
def test_mode_variances_and_sq_128(gs):
    cfg = dict(workloads.MID, gamma_shear=gs)
    kT, rho0 = cfg["kT"], cfg["rho0"]
    mu = 3 * kT
    lat = lbf.Lattice(**cfg, init="thermal")
    L = cfg["nx"]
    kk = torch.fft.fftfreq(L, device="cuda") * L
    kr = torch.sqrt(kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kk[None, None, :] ** 2)
    shells = [(0.5, 8), (8, 24), (24, 48), (48, 80), (80, 111)]
    var = []
    sq = torch.zeros((L, L, L), dtype=torch.float64, device="cuda")
    lat.step(100)
    nsnap = 90
    for s in range(nsnap):
        lat.step(10)
        m = lat.modes()
        v, rbar = neq_variances(m, rho0)
        var.append(v / (mu * rbar * W))
        sq += structure_factor(m[0])
        del m
    var = np.array(var)
    ratio = var.mean(axis=0)
    say(f"gamma_s={gs}: variance ratios min {ratio.min():.4f} max {ratio.max():.4f}")
    assert np.all(np.abs(ratio - 1) < 0.01), ratio
    S = sq / nsnap / (mu * rho0)
    for lo, hi in shells:
        sel = (kr >= lo) & (kr < hi)
        val = float(S[sel].mean())
        say(f"  S(q) shell [{lo},{hi}): {val:.4f}")
        assert abs(val - 1) < 0.01, (lo, hi, val)
    nb, sums = lat.check()
    assert nb == 0
    lat.close()


def shear_amplitude(mom, q):
    """A = (2 / Lz) sum_z <j_x>_{x,y}(z) sin(q z) and the x,y spread of j_x."""
    jx = mom[1].double()
    prof = jx.mean(dim=(1, 2))
    spread = float((jx - prof[:, None, None]).abs().max())
    z = torch.arange(jx.shape[0], device=jx.device, dtype=torch.float64)
    return float(2.0 / jx.shape[0] * (prof * torch.sin(q * z)).sum()), prof.cpu().numpy(), spread


@pytest.mark.parametrize("gs", [0.0, 0.5, 0.9])
def test_shear_wave_128_matches_exact_reduction(gs):
    U = 1e-3
    cfg = dict(workloads.MID, kT=0.0, gamma_shear=gs)
    L = cfg["nz"]
    q = 2 * np.pi / L
    f = workloads.shear_wave_fields(L, L, L, U)
    lat = lbf.Lattice(**cfg, init="fields", fields=torch.from_numpy(f))
    # the exact reduction: the same wave on 1 x 1 x L in FP64
    c1 = dict(cfg, nx=1, ny=1)
    p = oracle_params(c1)
    n = oracle.init(p, oracle.INIT_FIELDS, workloads.shear_wave_fields(1, 1, L, U).astype(np.float64))
    ts, amps = [], []
    t = 0
    for target in (0, 1, 200, 400, 600, 800, 1000):
        lat.step(target - t)
        n = oracle.run(p, n, t, target - t)
        t = target
        A, prof, spread = shear_amplitude(lat.moments(), q)
        want = oracle.moments(p, n)[1, :, 0, 0]
        err = np.abs(prof - want).max()
        assert spread < 1e-9, spread
        assert err < 1e-4 * U, (t, err)  # fp32 round-off over 1000 steps
        ts.append(t)
        amps.append(A)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 200
    slope = np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    nu_eff = -slope / q ** 2
    nu = th.nu_closed_form(gs)
    lam = abs(th.shear_eigenvalue(L, 1, th.mode_gammas(cfg["gamma_bulk"], gs, 0, 0), *oracle.tables()))
    say(f"gamma_s={gs}: nu_eff={nu_eff:.6f}, closed form {nu:.6f}, rel {nu_eff / nu - 1:+.2e}; "
        f"per-step decay {np.exp(slope):.10f} vs |lambda| {lam:.10f}")
    assert np.exp(slope) == pytest.approx(lam, abs=1e-6)
    if gs <= 0.5:
        assert nu_eff == pytest.approx(nu, rel=0.01)
    lat.close()


def test_viscosity_q0_limit_gamma09():
    """gamma_s = 0.9 carries a 7.6% O(q^2) lattice correction at L = 128;
    long boxes (n = 1, L = 512, 1024, 2048) extrapolated to q -> 0 recover
    Eq. shearviscosity within 1%."""
    gs, U = 0.9, 1e-3
    qs2, nus = [], []
    for L in (512, 1024, 2048):
        cfg = dict(nx=2, ny=2, nz=L, rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=gs,
                   gamma_odd=0.0, gamma_even=0.0, seed=0)
        q = 2 * np.pi / L
        lat = lbf.Lattice(**cfg, init="fields", fields=torch.from_numpy(workloads.shear_wave_fields(2, 2, L, U)))
        lat.step(300)
        t0 = lat.t
        A0, _, _ = shear_amplitude(lat.moments(), q)
        T = 3000
        lat.step(T)
        A1, _, _ = shear_amplitude(lat.moments(), q)
        qs2.append(q * q)
        nus.append(-np.log(A1 / A0) / T / (q * q))
        lat.close()
    qs2, nus = np.array(qs2), np.array(nus)
    # linear fit in q^2 over the three long waves
    nu0 = np.polyfit(qs2, nus, 1)[1]
    say(f"gamma_s=0.9: nu_eff {nus}, extrapolated {nu0:.5f}, closed form {th.nu_closed_form(gs):.5f}")
    assert nu0 == pytest.approx(th.nu_closed_form(gs), rel=0.01)


def test_stress_only_noise_matches_its_linear_theory():
    """With noise on the stress modes only (the earlier model the paper
    contrasts), every mode's stationary variance is that of the linearised
    update with noise on modes 4..9 alone (the discrete Lyapunov equation
    per wave vector, tests/lbtheory.py): the kinetic modes reach only 26-38%
    of mu rho w_k and, through streaming, the stress and conserved modes
    fall short too (31-51%).  The full detailed-balance collision keeps
    every mode at mu rho w_k.  Both checked to 1% on 32^3."""
    base = dict(nx=32, ny=32, nz=32, rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.5,
                gamma_odd=0.0, gamma_even=0.0, seed=77)
    mu = 3e-4
    c, a, e, w = oracle.tables()
    g = th.mode_gammas(0.5, 0.5, 0.0, 0.0)
    noisy = np.zeros(19, bool)
    noisy[4:10] = True
    theory = th.stationary_mode_variances((32, 32, 32), g, noisy, c, a, e, w)
    res = {}
    for mode in ("all", "stress_only"):
        lat = lbf.Lattice(**base, thermal_modes=mode, init="thermal")
        lat.step(200)
        acc = np.zeros(19)
        nsnap = 80
        for _ in range(nsnap):
            lat.step(5)
            v, rbar = neq_variances(lat.modes(), 1.0)
            acc += v / (mu * rbar * W)
        res[mode] = acc / nsnap
        lat.close()
    say(f"stress-only variance ratios: measured {res['stress_only'].round(4)}, theory {theory.round(4)}")
    assert np.all(np.abs(res["all"] - 1) < 0.01)
    np.testing.assert_allclose(res["stress_only"], theory, rtol=0.01)
    assert np.all(res["stress_only"][10:] < 0.4) and np.all(res["stress_only"][4:10] < 0.55)


@pytest.mark.parametrize("gb,gs", [(0.3, 0.5), (0.8, 0.0)])
def test_sound_wave_follows_linear_operator(gb, gs):
    """kT = 0 standing density wave rho = rho0 (1 + A sin(q z)) on 8 x 8 x 128:
    the GPU's density profile equals the exact FP64 1 x 1 x 128 reduction, and
    its Fourier amplitude follows the linearised one-step operator, whose
    q -> 0 limit is the sound speed c_s and the attenuation (4 nu / 3 +
    zeta / rho) / 2 of Eqs. shearviscosity and bulkviscosity."""
    A, L = 1e-4, 128
    cfg = dict(nx=8, ny=8, nz=L, rho0=1.0, kT=0.0, gamma_bulk=gb, gamma_shear=gs, gamma_odd=0.0,
               gamma_even=0.0, seed=0)
    q = 2 * np.pi / L
    f = workloads.density_wave_fields(8, 8, L, A)
    lat = lbf.Lattice(**cfg, init="fields", fields=torch.from_numpy(f))
    p = oracle_params(dict(cfg, nx=1, ny=1))
    n0 = oracle.init(p, oracle.INIT_FIELDS, workloads.density_wave_fields(1, 1, L, A).astype(np.float64))
    c, a, e, w = oracle.tables()
    z = np.arange(L)
    ph = np.exp(-1j * q * z)
    f0 = (n0[:, :, 0, 0] * ph[None, :]).sum(axis=1)
    Lop = th.one_step_operator([0, 0, q], th.mode_gammas(gb, gs, 0, 0), c, a, e, w)
    n, t = n0, 0
    for target in (1, 2, 100, 300, 600):
        lat.step(target - t)
        n = oracle.run(p, n, t, target - t)
        t = target
        # rho - rho0 from the modes gather (m_0), which keeps the deviation's precision
        drho = lat.modes()[0].double()
        prof = drho.mean(dim=(1, 2)).cpu().numpy()
        assert float((drho - drho.mean(dim=(1, 2))[:, None, None]).abs().max()) < 1e-12
        want = oracle.moments(p, n)[0, :, 0, 0] - cfg["rho0"]
        assert np.abs(prof - want).max() < 1e-4 * A, (t, np.abs(prof - want).max())
        rq = (prof * ph).sum()
        pred = (np.linalg.matrix_power(Lop, t) @ f0).sum()
        assert abs(rq - pred) < 1e-3 * abs(f0.sum()), (t, rq, pred)
    lat.close()
    lam = th.sound_eigenvalue(L, 1, th.mode_gammas(gb, gs, 0, 0), c, a, e, w)
    att = -np.log(abs(lam)) / q ** 2
    want_att = 0.5 * (4.0 / 3.0 * th.nu_closed_form(gs) + th.zeta_closed_form(gb))
    say(f"sound gb={gb} gs={gs}: attenuation {att:.5f} vs closed form {want_att:.5f}, "
        f"speed {abs(np.angle(lam)) / q:.5f} vs {np.sqrt(1 / 3):.5f}")
    assert att == pytest.approx(want_att, rel=0.02)
