"""The reduced (irreducible) storage of the expansions (the paper's closing
outlook: an irreducible representation cuts the Cartesian FMM's storage from
O(p^3) to O(p^2) per cell), checked on the CPU with the oracle's operators
before any kernel relies on it.

Derivatives of 1/r are harmonic, D_{k+2e_z} = -D_{k+2e_x} - D_{k+2e_y}, so
  - a multipole row M acts on every harmonic D like its fold F(M), which
    keeps only the components with m_z <= 1: component (a, b, 2j + r) adds
    (-1)^j C(j, i) M to component (a + 2i, b + 2(j - i), r);
  - a local row L formed by M2L inherits the identity, so its components
    with n_z <= 1 determine all others:
    L_(a, b, 2j + r) = (-1)^j sum_i C(j, i) L_(a + 2i, b + 2(j - i), r).
What the reduced storage needs: F(M2M(M)) = F(M2M(lift(F(M)))) (M2M may run
on folded rows lifted with zeros), M2L outputs and L2L results are harmonic
(so L2L may run on rebuilt rows and keep the reduced part), and L2P of the
rebuilt row equals L2P of the full row."""
from math import comb

import numpy as np
import pytest


def _mi(orc, p):
    return [tuple(orc.multi_index(i)) for i in range(orc.nterms(p))]


def fold(orc, M, p):
    """F(M): the components with m_z <= 1 (others zero) of the full row M"""
    F = np.zeros_like(M)
    for i, (a, b, c) in enumerate(_mi(orc, p)):
        j, r = divmod(c, 2)
        for k in range(j + 1):
            F[orc.index(a + 2 * k, b + 2 * (j - k), r)] += (-1) ** j * comb(j, k) * M[i]
    return F


def restrict(orc, L, q):
    """the components with n_z <= 1 (others zero)"""
    return np.array([v if c <= 1 else 0.0 for v, (a, b, c) in zip(L, _mi(orc, q))])


def rebuild(orc, Lr, q):
    """every component from those with n_z <= 1"""
    L = np.zeros_like(Lr)
    for i, (a, b, c) in enumerate(_mi(orc, q)):
        j, r = divmod(c, 2)
        L[i] = (-1) ** j * sum(comb(j, k) * Lr[orc.index(a + 2 * k, b + 2 * (j - k), r)] for k in range(j + 1))
    return L


@pytest.mark.parametrize("p,s", [(4, 0), (8, 1), (10, 2), (7, 3)])
def test_fold_acts_like_the_row_on_harmonic_tensors(orc, p, s):
    rng = np.random.default_rng(p + 10 * s)
    M = rng.standard_normal(orc.nterms(p))
    M[:orc.nterms(s - 1)] = 0.0
    F = fold(orc, M, p)
    assert all(F[i] == 0.0 for i, (a, b, c) in enumerate(_mi(orc, p)) if c > 1)
    for _ in range(3):
        x = rng.standard_normal(3) * 3.0
        D = orc.dtensor(p, x)
        assert abs(F @ D - M @ D) <= 1e-12 * np.abs(M * D).sum()
    # the fold loses only what no harmonic tensor sees: the potential and
    # field of the row and its fold agree at any far point
    zA = np.zeros(3)
    for _ in range(3):
        x = rng.standard_normal(3) * 4.0
        a = orc.m2p(p, s, zA, M, x)
        b = orc.m2p(p, s, zA, F, x)
        assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0]) + 1e-15 and np.allclose(a[1], b[1], rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("p,s", [(4, 0), (8, 1), (10, 2), (7, 3)])
def test_m2m_commutes_with_the_fold(orc, p, s):
    rng = np.random.default_rng(3 * p + s)
    M = rng.standard_normal(orc.nterms(p))
    M[:orc.nterms(s - 1)] = 0.0
    for _ in range(3):
        zc = rng.standard_normal(3) * 0.1
        zp = zc + rng.choice([-0.25, 0.25], 3)
        a = fold(orc, orc.m2m(p, zc, M, zp), p)
        b = fold(orc, orc.m2m(p, zc, fold(orc, M, p), zp), p)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        # and the folded row's multipole orders below s stay zero
        assert np.all(b[:orc.nterms(s - 1)] == 0.0)


@pytest.mark.parametrize("p,s", [(4, 0), (8, 1), (10, 2), (7, 3)])
def test_locals_are_rebuilt_from_their_reduced_part(orc, p, s):
    """M2L output (Eq. 8 with the truncation |m| <= p - |n|), its L2L shift
    and the sum of several are harmonic: the n_z <= 1 part rebuilds them"""
    rng = np.random.default_rng(5 * p + s)
    q = p - s
    zB = np.zeros(3)
    L = np.zeros(orc.nterms(q))
    for _ in range(3):
        M = rng.standard_normal(orc.nterms(p))
        M[:orc.nterms(s - 1)] = 0.0
        zA = rng.standard_normal(3) * 0.2 + np.array([2.5, -1.0, 0.7])
        L += orc.m2l(p, s, zA, M, zB)
    R = rebuild(orc, restrict(orc, L, q), q)
    assert np.abs(R - L).max() <= 1e-12 * np.abs(L).max()
    zC = rng.choice([-0.25, 0.25], 3)
    Lc = orc.l2l(p, s, zB, L, zC)
    assert np.abs(rebuild(orc, restrict(orc, Lc, q), q) - Lc).max() <= 1e-12 * np.abs(Lc).max()
    # L2L of the rebuilt parent keeps the child's reduced part
    Lc2 = orc.l2l(p, s, zB, R, zC)
    assert np.abs(restrict(orc, Lc2, q) - restrict(orc, Lc, q)).max() <= 1e-12 * np.abs(Lc).max()
    # and L2P of the rebuilt row is L2P of the row
    x = zC + rng.standard_normal(3) * 0.1
    a, b = orc.l2p(p, s, zB, L, x), orc.l2p(p, s, zB, R, x)
    assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0]) and np.allclose(a[1], b[1], rtol=1e-11, atol=0)


def test_a_row_that_is_not_harmonic_is_not_rebuilt(orc):
    """the rebuild is no identity on arbitrary rows (the check above is not
    vacuous): a random local row differs from its rebuilt reduced part"""
    rng = np.random.default_rng(1)
    L = rng.standard_normal(orc.nterms(6))
    assert np.abs(rebuild(orc, restrict(orc, L, 6), 6) - L).max() > 0.1
