"""Pins of the oracle's angle set (paper section 3.2) against facts that do not come
from the oracle: exact moment conditions, closed forms solved by hand, the cube
symmetry group, and exact rational arithmetic."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

N_MUS = (2, 4, 6, 8, 10, 12)


@pytest.mark.parametrize("n_mu", N_MUS)
def test_counts_and_unit_vectors(oracle_mod, n_mu):
    mu, w = oracle_mod.quadrature(n_mu)
    # section 3.2: n_a = n_mu (n_mu + 2) rays in 3D, identical octants
    assert mu.shape == (n_mu * (n_mu + 2), 3)
    assert np.allclose(np.sum(mu * mu, axis=1), 1.0, atol=1e-15)
    assert np.all(w > 0)
    per = len(w) // 8
    for o in range(8):
        sg = np.array([-1.0 if (o >> q) & 1 else 1.0 for q in range(3)])
        blk = mu[o * per:(o + 1) * per]
        assert np.all(np.sign(blk) == sg)
        assert np.array_equal(np.abs(blk), np.abs(mu[:per]))
        assert np.array_equal(w[o * per:(o + 1) * per], w[:per])


@pytest.mark.parametrize("n_mu", N_MUS)
def test_moments(oracle_mod, n_mu):
    mu, w = oracle_mod.quadrature(n_mu)
    assert abs(np.sum(w) - 1.0) < 1e-15
    for q in range(3):
        assert abs(np.sum(w * mu[:, q])) < 1e-16          # odd moments vanish
        assert abs(np.sum(w * mu[:, q] ** 3)) < 1e-16
        # K = J/3 for an isotropic field (section 3.2, the n_mu = 2 remark and eq. Ksum)
        assert abs(np.sum(w * mu[:, q] ** 2) - 1.0 / 3.0) < 1e-15
        for r in range(q + 1, 3):
            assert abs(np.sum(w * mu[:, q] * mu[:, r])) < 1e-16
    if n_mu >= 4:
        for p in range(2, n_mu // 2 + 1):
            # exact even moments of the sphere: <mu^2p> = 1/(2p+1)
            assert abs(np.sum(w * mu[:, 0] ** (2 * p)) - 1.0 / (2 * p + 1)) < 2e-15


@pytest.mark.parametrize("n_mu", N_MUS)
def test_cube_symmetry(oracle_mod, n_mu):
    """Invariance under all 48 rotations/reflections of the cube (section 3.2)."""
    mu, w = oracle_mod.quadrature(n_mu)
    key = {tuple(np.round(m, 13)): wt for m, wt in zip(mu, w)}
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            t = mu[:, perm] * np.array(signs)
            for m, wt in zip(t, w):
                k = tuple(np.round(m, 13))
                assert k in key and abs(key[k] - wt) < 1e-15


def test_two_stream_set(oracle_mod):
    """n_mu = 2: one ray per octant along the cube diagonal, K_ij = delta_ij J/3."""
    mu, w = oracle_mod.quadrature(2)
    assert np.allclose(np.abs(mu), 1.0 / np.sqrt(3.0), atol=1e-16)
    assert np.allclose(w, 1.0 / 8.0, atol=0)


def test_lq4_closed_form(oracle_mod):
    """n_mu = 4: per octant the 3 permutations of (mu1, mu1, mu2), weights 1/24,
    2 mu1^2 + mu2^2 = 1 and <mu_x^4> = 1/5 give 6 a^2 - 4 a + 2/5 = 0 for a = mu1^2;
    the root below 1/3 is a = (4 - sqrt(6.4))/12, mu1 = 0.3500212, mu2 = 0.8688903."""
    a = (4.0 - np.sqrt(6.4)) / 12.0
    mu1, mu2 = np.sqrt(a), np.sqrt(1.0 - 2.0 * a)
    mu, w = oracle_mod.quadrature(4)
    oct0 = np.abs(mu[:3])
    assert np.allclose(np.sort(oct0, axis=1), [[mu1, mu1, mu2]] * 3, atol=2e-15)
    assert np.allclose(w, 1.0 / 24.0, atol=1e-17)
    assert abs(mu1 - 0.3500212) < 5e-8 and abs(mu2 - 0.8688903) < 5e-8


def _exact_conditions(n_mu, a):
    """Solve the class weights in exact rationals from p = 0, 2..m-1 and return the
    residual of the p = m condition."""
    m = n_mu // 2
    cls = [(i, j, k) for i in range(1, m + 1) for j in range(i, m + 1) for k in range(j, m + 1)
           if i + j + k == m + 2]
    step = Fraction(2) * (1 - 3 * a) / (n_mu - 2)
    lev = [a + i * step for i in range(m)]

    def mom(c, p):
        return sum(lev[t[0] - 1] ** p for t in set(itertools.permutations(c)))

    ps = [0] + list(range(2, m))
    A = [[mom(c, p) for c in cls] for p in ps]
    b = [Fraction(1, 2 * p + 1) for p in ps]
    n = len(cls)
    for col in range(n):  # Gauss-Jordan in rationals
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                fct = A[r][col] / A[col][col]
                A[r] = [x - fct * y for x, y in zip(A[r], A[col])]
                b[r] -= fct * b[col]
    wc = [b[i] / A[i][i] for i in range(n)]
    return sum(wc[i] * mom(c, m) for i, c in enumerate(cls)) - Fraction(1, 2 * m + 1), wc


def test_lq8_exact_rational(oracle_mod):
    """n_mu = 8: mu1^2 = 1/21 satisfies every even-moment condition exactly (checked
    in rational arithmetic), so the oracle's mu1 must be 1/sqrt(21)."""
    resid, wc = _exact_conditions(8, Fraction(1, 21))
    assert resid == 0 and all(x > 0 for x in wc)
    mu, w = oracle_mod.quadrature(8)
    assert abs(np.min(np.abs(mu)) - 1.0 / np.sqrt(21.0)) < 1e-15
    # class weights (per octant normalised to 1) equal the exact rationals
    per = np.unique(np.round(w[:10] * 8, 14))
    assert np.allclose(np.sort(per), np.sort([float(x) for x in wc]), atol=1e-14)


def test_lq_literature_values(oracle_mod):
    """mu1 of the level-symmetric sets as tabulated in the transport literature
    (LQ_n: 0.3500212, 0.2666355, 0.2182179, 0.1893213, 0.1672126)."""
    ref = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 10: 0.1893213, 12: 0.1672126}
    for n, v in ref.items():
        mu, _ = oracle_mod.quadrature(n)
        assert abs(np.min(np.abs(mu)) - v) < 2e-7
