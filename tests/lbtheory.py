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


def load_table2():
    """[(k, polynomial source, Fraction w_k)] from Table II."""
    rows = []
    with open(os.path.join(GOLDEN, "table2_d3q19.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, poly, w = [s.strip() for s in line.split("|")]
            rows.append((int(k), poly, Fraction(w)))
    return rows


def table2_matrix(c):
    """e[k, i] evaluated exactly (Fractions) from the Table II polynomials
    for the velocity list c (19 x 3 integers)."""
    rows = load_table2()
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
    """19x19 linearised collide-and-push operator for a plane wave
    exp(i q.r): L = diag(exp(-i q.c_i)) * Minv diag(gamma) M with M = e
    (m = M n) and Minv[i, k] = a_i e_ki / w_k."""
    M = np.asarray(e, dtype=float)
    Minv = (np.asarray(a)[:, None] * M.T) / np.asarray(w)[None, :]
    C = Minv @ np.diag(gammas) @ M
    phase = np.exp(-1j * (np.asarray(c, dtype=float) @ np.asarray(q_vec, dtype=float)))
    return phase[:, None] * C


def mode_gammas(gb, gs, go, ge):
    g = np.ones(19)
    g[4] = gb
    g[5:10] = gs
    g[10:16] = go
    g[16:19] = ge
    return g


def shear_eigenvalue(L, n, gammas, c, a, e, w):
    """Eigenvalue of the transverse-momentum (j_x, wave vector along z)
    mode: the eigenvector with the largest overlap with j_x."""
    q = 2 * np.pi * n / L
    Lop = one_step_operator([0, 0, q], gammas, c, a, e, w)
    vals, vecs = np.linalg.eig(Lop)
    jx = np.asarray(c, dtype=float)[:, 0]
    best = np.argmax(np.abs(jx @ vecs) / np.linalg.norm(vecs, axis=0))
    return vals[best]


def sound_eigenvalue(L, n, gammas, c, a, e, w):
    """Eigenvalue of the forward sound mode (wave vector along z): the
    eigenvector with the largest density + j_z overlap, positive frequency."""
    q = 2 * np.pi * n / L
    Lop = one_step_operator([0, 0, q], gammas, c, a, e, w)
    vals, vecs = np.linalg.eig(Lop)
    cz = np.asarray(c, dtype=float)[:, 2]
    ov = (np.abs(np.ones(19) @ vecs) + np.abs(cz @ vecs)) / np.linalg.norm(vecs, axis=0)
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
