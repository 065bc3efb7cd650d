"""Test-side theory helpers: golden-fixture loaders, an independent pure-Python
Philox4x32-10, the linearised one-step operator of the D3Q19 update in
Fourier space, and the statistics used by the stationary-law pins.

None of this is product code and none of it calls the GPU library.
"""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CS2 = 1.0 / 3.0


# ---------------------------------------------------------------- fixtures
def load_weights():
    """{|c|^2: (count, Fraction weight)}, cs2 (Sec. II)."""
    out, cs2 = {}, None
    with open(os.path.join(GOLDEN, "d3q19_weights.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0] == "cs2":
                cs2 = Fraction(parts[1])
            else:
                out[int(parts[0])] = (int(parts[1]), Fraction(parts[2]))
    return out, cs2


def load_table2(name="table2_d3q19.txt"):
    """[(k, polynomial source, Fraction w_k)] from Table II (or, with
    name="table1_d2q9.txt", from Table I)."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, poly, w = [s.strip() for s in line.split("|")]
            rows.append((int(k), poly, Fraction(w)))
    return rows


def table2_matrix(c, name="table2_d3q19.txt"):
    """e[k, i] evaluated exactly (Fractions) from the Table II polynomials
    (or those of another fixture) for the velocity list c (q x 3 integers)."""
    rows = load_table2(name)
    e = [[None] * len(c) for _ in rows]
    for k, poly, _ in rows:
        for i, (cx, cy, cz) in enumerate(c):
            cx, cy, cz = Fraction(int(cx)), Fraction(int(cy)), Fraction(int(cz))
            c2 = cx * cx + cy * cy + cz * cz
            e[k][i] = Fraction(eval(poly, {"__builtins__": {}},
                                    {"cx": cx, "cy": cy, "cz": cz, "c2": c2}))
    return e


# ---------------------------------------------------------------- Philox
M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10_py(ctr, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC'11), written with Python
    integers: each round multiplies counter words 0 and 2 by the two
    multipliers, and the next counter is (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2),
    hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); the key advances by the two Weyl
    constants between rounds."""
    x0, x1, x2, x3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & MASK, p1 & MASK, \
                         ((p0 >> 32) ^ x3 ^ k1) & MASK, p0 & MASK
    return [x0, x1, x2, x3]


def chunks24_py(seed, site, t, stream, n):
    """24-bit chunks of the (seed, site, t, stream) word stream, built as one
    big integer per three words."""
    nwords = 3 * ((n + 3) // 4)
    words = []
    call = 0
    while len(words) < nwords:
        words += philox4x32_10_py(
            [site, t & MASK, (stream << 16) | call, t >> 32],
            [seed & MASK, seed >> 32])
        call += 1
    out = []
    for c in range(n):
        w = words[3 * (c // 4): 3 * (c // 4) + 3]
        big = (w[0] << 64) | (w[1] << 32) | w[2]
        out.append((big >> (72 - 24 * (c % 4))) & 0xFFFFFF)
    return out


# ---------------------------------------------------------------- linear operator
def one_step_operator(q_vec, gammas, c, a, e, w):
    """q x q linearised collide-and-push operator for a plane wave
    exp(i q.r): L = diag(exp(-i q.c_i)) * Minv diag(gamma) M with M = e
    (m = M n) and Minv[i, k] = a_i e_ki / w_k."""
    M = np.asarray(e, dtype=float)
    Minv = (np.asarray(a)[:, None] * M.T) / np.asarray(w)[None, :]
    C = Minv @ np.diag(gammas) @ M
    phase = np.exp(-1j * (np.asarray(c, dtype=float) @ np.asarray(q_vec, dtype=float)))
    return phase[:, None] * C


def mode_gammas(gb, gs, go, ge, q=19):
    """Per-mode rates in table order: D3Q19 (q = 19) k = 4 bulk, 5..9 shear,
    10..15 odd, 16..18 even; D2Q9 (q = 9) k = 3 bulk, 4..5 shear, 6..7 odd,
    8 even; conserved modes 1."""
    g = np.ones(q)
    if q == 19:
        g[4] = gb
        g[5:10] = gs
        g[10:16] = go
        g[16:19] = ge
    else:
        g[3] = gb
        g[4:6] = gs
        g[6:8] = go
        g[8] = ge
    return g


def shear_eigenvalue(L, n, gammas, c, a, e, w, axis=2):
    """Eigenvalue of the transverse-momentum (j_x, wave vector along z, or
    along `axis`) mode: the eigenvector with the largest overlap with j_x."""
    q = 2 * np.pi * n / L
    qv = [0.0, 0.0, 0.0]
    qv[axis] = q
    Lop = one_step_operator(qv, gammas, c, a, e, w)
    vals, vecs = np.linalg.eig(Lop)
    jx = np.asarray(c, dtype=float)[:, 0]
    best = np.argmax(np.abs(jx @ vecs) / np.linalg.norm(vecs, axis=0))
    return vals[best]


def sound_eigenvalue(L, n, gammas, c, a, e, w, axis=2):
    """Eigenvalue of the forward sound mode (wave vector along z, or along
    `axis`): the eigenvector with the largest density + longitudinal
    momentum overlap, positive frequency."""
    q = 2 * np.pi * n / L
    qv = [0.0, 0.0, 0.0]
    qv[axis] = q
    Lop = one_step_operator(qv, gammas, c, a, e, w)
    vals, vecs = np.linalg.eig(Lop)
    cz = np.asarray(c, dtype=float)[:, axis]
    ov = (np.abs(np.ones(len(cz)) @ vecs) + np.abs(cz @ vecs)) / np.linalg.norm(vecs, axis=0)
    order = np.argsort(-ov)
    for idx in order[:4]:
        if np.angle(vals[idx]) < 0:  # exp(-i w) convention of the push
            return vals[idx]
    return vals[order[0]]


def nu_closed_form(gs):
    """Kinematic shear viscosity eta/rho, Eq. shearviscosity (h = 1)."""
    return CS2 * (1 + gs) / (2 * (1 - gs))


def zeta_closed_form(gb, d=3):
    """Bulk viscosity zeta/rho, Eq. bulkviscosity (h = 1)."""
    return CS2 / d * (1 + gb) / (1 - gb)


def extrapolate_q0(qs2, vals):
    """Fit vals = v0 + v1 q^2 + v2 q^4 and return v0."""
    A = np.vstack([np.ones_like(qs2), qs2, qs2 ** 2]).T
    coef, *_ = np.linalg.lstsq(A, vals, rcond=None)
    return coef[0]


# ---------------------------------------------------------------- stationary law of the linear update
def stationary_mode_variances(dims, gammas, noisy, c, a, e, w, structure_factor=False, batch=2048,
                              doublings=16):
    """Equal-time per-site mode variances of the linearised fluctuating
    update on a periodic box, in units of mu rho w_k.

    For small noise the deviation from rest evolves, per wave vector q, as
    x(t + 1) = S(q) (C x(t) + xi(t)) with C = Minv diag(gamma) M the
    collision, S(q) = diag(exp(-i q.c_i)) the push and xi the collision
    noise: sqrt(w_k (1 - gamma_k^2)) r_k on the modes flagged in `noisy`
    (mu rho = 1), none elsewhere.  The stationary covariance solves the
    discrete Lyapunov equation X = A X A^H + S B S^H with A = S C and
    B = Minv diag(noise variances) Minv^T; it is summed here as
    X = sum_n A^n (S B S^H) A^nH by repeated squaring.  The per-site
    covariance is the average of X(q) over the box's wave vectors, and
    the mode variances are the diagonal of M (that average) M^T, divided by
    w_k.  Conserved modes carry no noise, so at q = 0 they do not
    fluctuate: the result for k <= d is the variance about the lattice
    mean, as measured.

    With every non-conserved mode noisy (the detailed-balance collision,
    Sec. IV) the result is 1 for the non-conserved modes and 1 - 1/N for
    the conserved ones (the q = 0 part is missing).  With noise on the
    stress modes only (the earlier model the paper contrasts) it is not.

    With structure_factor=True also returns {|q|^2: mean S(q) / (mu rho)}
    over the nonzero wave vectors (the density-density correlation of mode
    0, Eq. mpeos's mu rho for the detailed-balance collision)."""
    M = np.asarray(e, dtype=float)
    q = M.shape[0]
    wv = np.asarray(w, dtype=float)
    g = np.asarray(gammas, dtype=float)
    Minv = (np.asarray(a)[:, None] * M.T) / wv[None, :]
    C = Minv @ np.diag(g) @ M
    nv = np.where(np.asarray(noisy, bool), wv * (1.0 - g * g), 0.0)
    B = Minv @ np.diag(nv) @ Minv.T
    cf = np.asarray(c, dtype=float)
    dims = tuple(int(v) for v in dims)
    grids = np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in dims], indexing="ij")
    qs = np.stack([gr.ravel() for gr in grids], axis=1)  # (N, 3)
    N = qs.shape[0]
    acc = np.zeros((q, q))
    sq = {}
    for s0 in range(0, N, batch):
        qv = qs[s0:s0 + batch]
        ph = np.exp(-1j * (qv @ cf.T))  # (b, q)
        A = ph[:, :, None] * C[None, :, :]
        X = ph[:, :, None] * B[None, :, :] * ph.conj()[:, None, :]
        Ap = A
        for _ in range(doublings):  # 2^doublings terms: far past the slowest decay of a box <= 64
            X = X + Ap @ X @ np.conj(np.swapaxes(Ap, 1, 2))
            Ap = Ap @ Ap
        acc += X.real.sum(axis=0)
        if structure_factor:
            s00 = np.einsum("i,bij,j->b", M[0], X, M[0]).real
            q2 = np.round((qv * qv).sum(axis=1), 12)
            for k2, v in zip(q2, s00):
                if k2 > 0:
                    sq.setdefault(k2, []).append(v)
    acc /= N
    mv = np.diag(M @ acc @ M.T) / wv
    if structure_factor:
        return mv, {k2: float(np.mean(v)) for k2, v in sorted(sq.items())}
    return mv


# ---------------------------------------------------------------- statistics
def neq_modes(modes, rho0):
    """Non-equilibrium part of the unscaled modes, (19, ...) array of m_k of
    n - a rho0.  For k >= 4 subtracts m_k^eq(rho, j) from the quadratic
    equilibrium; k <= 3 are returned about their lattice mean."""
    m = np.array(modes, dtype=np.float64)
    rho = rho0 + m[0]
    jx, jy, jz = m[1], m[2], m[3]
    eq = np.zeros_like(m)
    eq[4] = (jx * jx + jy * jy + jz * jz) / rho
    eq[5] = (2 * jx * jx - jy * jy - jz * jz) / rho
    eq[6] = (jy * jy - jz * jz) / rho
    eq[7] = jx * jy / rho
    eq[8] = jy * jz / rho
    eq[9] = jz * jx / rho
    out = m - eq
    for k in range(4):
        out[k] = m[k] - m[k].mean()
    return out


# ---------------------------------------------------------------- macroscopic random stress
def box_random_stress(m_before, m_after, rho0, gammas, c, a, e, w):
    """Box sum of the random stress R_ab that one collision adds (Sec. IV),
    from the gathered modes ((q, ...) of n - a rho0) at t and at t + 1.

    Streaming moves every population to another site but keeps the box total
    of each direction, so the box sum of each mode after the step equals the
    box sum of the post-collision modes.  Subtracting the deterministic part
    m^eq + gamma_k (m - m^eq) of the modes at t leaves sum_r R_k(r) for the
    non-conserved modes; the back-transform dn_i = a_i sum_k e_ki R_k / w_k
    turns them into population changes, whose second velocity moment is the
    stress tensor R_ab (kinetic modes drop out: they are orthogonal to every
    polynomial of degree <= 2)."""
    c = np.asarray(c)
    d = int(np.count_nonzero(np.abs(c).sum(axis=0)))
    q = len(c)
    mb = np.asarray(m_before, dtype=np.float64).reshape(q, -1)
    ma = np.asarray(m_after, dtype=np.float64).reshape(q, -1)
    eq = mb - neq_modes_any(mb, rho0, c, a, e)
    eq[: 1 + d] = 0.0  # conserved modes: gamma = 1, nothing to subtract
    g = np.asarray(gammas)[:, None]
    post = np.where(np.arange(q)[:, None] <= d, mb, eq + g * (mb - eq))
    Rk = ma.sum(axis=1) - post.sum(axis=1)
    Rk[: 1 + d] = 0.0
    dn = np.asarray(a) * (np.asarray(e).T @ (Rk / np.asarray(w)))
    cc = c[:, :d].astype(float)
    return np.einsum("i,ia,ib->ab", dn, cc, cc)


def macroscopic_stress(R, gb, gs, d=3):
    """Random stress on the hydrodynamic level, Q = -Rbar/(1 - gs) -
    delta tr(R)/(d (1 - gb)) with Rbar the traceless part of R (Sec. V)."""
    tr = np.trace(R)
    dev = R - tr / d * np.eye(d)
    return -dev / (1 - gs) - tr / (d * (1 - gb)) * np.eye(d)


def macro_stress_covariance(kT, eta, zeta, d=3):
    """<Q_ab Q_cd> per unit volume and time step, Eq. macrostressfluct with
    b = h = 1 and m_p cs^2 = kT (Eq. mpeos); returned as a (d,)*4 array."""
    I = np.eye(d)
    return 2 * kT * ((zeta - 2 * eta / d) * np.einsum("ab,cd->abcd", I, I)
                     + eta * (np.einsum("ac,bd->abcd", I, I) + np.einsum("ad,bc->abcd", I, I)))


# ---------------------------------------------------------------- any lattice
def equilibrium_fields(rho, j, c, a):
    """n_i^eq(rho, u = j / rho) of Eq. derived_equil_distrib with c_s^2 = 1/3
    for whole fields: rho (N,), j (d, N) -> (q, N)."""
    c = np.asarray(c, dtype=float)[:, : len(j)]
    u = np.asarray(j) / rho
    uc = c @ u
    uu = (u * u).sum(axis=0)
    return np.asarray(a)[:, None] * rho * (1 + uc / CS2 + uc * uc / (2 * CS2 ** 2) - uu / (2 * CS2))


def neq_modes_any(modes, rho0, c, a, e):
    """neq_modes for any velocity set: m_k - m_k^eq for the non-conserved
    modes k > d (m^eq projected from the equilibrium populations), and the
    conserved modes about their lattice mean.  modes: (q, ...) of n - a rho0."""
    m = np.array(modes, dtype=np.float64)
    shp = m.shape
    m = m.reshape(len(m), -1)
    d = int(np.count_nonzero(np.abs(np.asarray(c)).sum(axis=0)))
    rho = rho0 + m[0]
    neq = equilibrium_fields(rho, m[1:1 + d], c, a)
    meq = np.asarray(e) @ (neq - np.asarray(a)[:, None] * rho0)
    out = m - meq
    for k in range(1 + d):
        out[k] = m[k] - m[k].mean()
    return out.reshape(shp)
