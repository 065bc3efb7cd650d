"""Pins of the oracle's lattice tables against what the paper prints:
the D3Q19 weights (Sec. II), the moment conditions on the weights (Eqs.
wi0-wi4 with equilcond2-equilcond3), Table II's polynomials and w_k, and the
explicitly written orthonormal hydrodynamic vectors of Sec. III."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import lbtheory as th


@pytest.fixture(scope="module")
def tabs():
    return oracle.tables()


def test_velocity_set_is_d3q19(tabs):
    c, a, e, w = tabs
    want = {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(x * x for x in v) <= 2}
    assert len(want) == 19
    assert {tuple(map(int, v)) for v in c} == want
    # opposite pairs: i+1 for odd i, i-1 for even i > 0
    for i in range(1, 19):
        o = i + 1 if i % 2 else i - 1
        assert tuple(-c[i]) == tuple(c[o])


def test_weights_match_paper(tabs):
    c, a, e, w = tabs
    golden, cs2 = th.load_weights()
    for c2, (count, wt) in golden.items():
        idx = [i for i in range(19) if int((c[i] ** 2).sum()) == c2]
        assert len(idx) == count
        for i in idx:
            assert a[i] == pytest.approx(float(wt), abs=1e-16)
    assert float(cs2) == pytest.approx(1.0 / 3.0)


def test_weight_moment_conditions():
    """Eqs. wi0-wi4 and equilcond2-equilcond3 in exact rational arithmetic:
    sum a = 1, odd moments vanish, sigma_2 = c_s^2 = 1/3, sigma_4 = sigma_2^2,
    kappa_4 = 0."""
    golden, cs2 = th.load_weights()
    c = [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(x * x for x in v) <= 2]
    a = [golden[sum(x * x for x in v)][1] for v in c]
    assert sum(a) == 1
    for al in range(3):
        assert sum(ai * ci[al] for ai, ci in zip(a, c)) == 0
        for be in range(3):
            s2 = sum(ai * ci[al] * ci[be] for ai, ci in zip(a, c))
            assert s2 == (cs2 if al == be else 0)
            for ga in range(3):
                assert sum(ai * ci[al] * ci[be] * ci[ga] for ai, ci in zip(a, c)) == 0
    sigma4 = cs2 * cs2
    for al, be, ga, de in itertools.product(range(3), repeat=4):
        m4 = sum(ai * ci[al] * ci[be] * ci[ga] * ci[de] for ai, ci in zip(a, c))
        iso = sigma4 * ((al == be) * (ga == de) + (al == ga) * (be == de) + (al == de) * (be == ga))
        assert m4 == iso  # kappa_4 = 0


def test_table2_polynomials_and_lengths(tabs):
    """The oracle's e_ki equal Table II's polynomials evaluated exactly, and
    its w_k equal the printed third column."""
    c, a, e, w = tabs
    ex = th.table2_matrix(c)
    rows = th.load_table2()
    for k, _, wk in rows:
        for i in range(19):
            assert e[k, i] == float(ex[k][i])
        assert w[k] == pytest.approx(float(wk), rel=1e-15)
        # w_k recomputed exactly from the golden polynomials and weights
        golden, _ = th.load_weights()
        aw = [golden[int((ci ** 2).sum())][1] for ci in c]
        assert sum(aw[i] * ex[k][i] ** 2 for i in range(19)) == wk


def test_table2_orthogonality_exact(tabs):
    """sum_i a_i e_ki e_li = w_k delta_kl (Eq. orthogonality after Eq.
    evectors_orthonormal), exactly, and 207 non-zero entries."""
    c, a, e, w = tabs
    ex = th.table2_matrix(c)
    golden, _ = th.load_weights()
    aw = [golden[int((ci ** 2).sum())][1] for ci in c]
    for k in range(19):
        for l in range(19):
            s = sum(aw[i] * ex[k][i] * ex[l][i] for i in range(19))
            if k != l:
                assert s == 0, (k, l)
    assert sum(1 for k in range(19) for i in range(19) if ex[k][i] != 0) == 207


def test_text_orthonormal_vectors_match_table(tabs):
    """Sec. III writes the hydrodynamic and stress vectors out in closed form;
    they must equal sqrt(a_i / w_k) e_ki from Table II for k = 0..9 (with the
    (c_y^2 - c_z^2) shear vector as k = 6 and cyclic permutations)."""
    c, a, e, w = tabs
    cs2, d = 1.0 / 3.0, 3
    ehat = np.sqrt(a[None, :] / w[:, None]) * e
    cx, cy, cz = c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float)
    c2 = cx ** 2 + cy ** 2 + cz ** 2
    sa = np.sqrt(a)
    text = {
        0: sa,
        1: np.sqrt(a / cs2) * cx, 2: np.sqrt(a / cs2) * cy, 3: np.sqrt(a / cs2) * cz,
        4: (1 / cs2) * np.sqrt(a / (2 * d)) * (c2 - d * cs2),
        5: (1 / cs2) * np.sqrt(a / (2 * d * (d - 1))) * (d * cx ** 2 - c2),
        6: sa / (2 * cs2) * (cy ** 2 - cz ** 2),
        7: sa / cs2 * cx * cy, 8: sa / cs2 * cy * cz, 9: sa / cs2 * cz * cx,
    }
    for k, v in text.items():
        np.testing.assert_allclose(ehat[k], v, atol=1e-15, err_msg=f"mode {k}")
    # completeness of the orthonormal basis
    np.testing.assert_allclose(ehat @ ehat.T, np.eye(19), atol=1e-14)
    np.testing.assert_allclose(ehat.T @ ehat, np.eye(19), atol=1e-14)
